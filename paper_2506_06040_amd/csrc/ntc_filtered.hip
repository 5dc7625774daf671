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
#ifndef NTC_FILT_TRI_SUBS  // 64-pixel sub-spans per staged span of the trilinear decode
#define NTC_FILT_TRI_SUBS 16
#endif
#ifndef NTC_FILT_ANI_SUBS  // and of the anisotropic decode
#define NTC_FILT_ANI_SUBS 4
#endif

// Mip m of level k as a sampling table entry (clamp to edge).
__device__ __forceinline__ TabLevel mip_level(const FilterArgs &f, int k, int m) {
  const MipArgs &M = f.mip[k][m];
  TabLevel L;
  L.fw = M.fw;
  L.fh = M.fh;
  L.cx = f.sx[k] - 0.5f;
  L.cy = f.sy[k] - 0.5f;
  L.wm2 = M.fw - 2.0f;
  L.hm2 = M.fh - 2.0f;
  L.w = M.w;
  L.h = M.h;
  L.bw = M.bw;
  L.bc1 = M.bc1;
  return L;
}

__device__ __forceinline__ float uniform_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
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
  float inv;  // 1 / (n + 1)
};

// The part of the selection that does not depend on the level's mip count:
// the unclamped level of detail and, for anisotropic filtering, the tap
// count and the major axis, from the footprint on a level of w0 x h0 texels.
struct LodBase {
  float lod;
  int n;
  float du, dv;
  float inv;  // 1 / (n + 1)
};

template <int FILTER>
__device__ __forceinline__ LodBase lod_base(const FilterArgs &f, float w0, float h0, float4 d) {
  LodBase b;
  // squared footprint axes in mip-0 texels, each operation rounded once
  const float ax = __fmul_rn(d.x, w0), bx = __fmul_rn(d.y, h0);
  const float ay = __fmul_rn(d.z, w0), by = __fmul_rn(d.w, h0);
  const float px2 = __fadd_rn(__fmul_rn(ax, ax), __fmul_rn(bx, bx));
  const float py2 = __fadd_rn(__fmul_rn(ay, ay), __fmul_rn(by, by));
  if (FILTER == 1) {
    b.lod = 0.5f * __log2f(fmaxf(px2, py2));
    b.n = 1;
    b.du = 0.0f;
    b.dv = 0.0f;
    b.inv = 0.5f;
  } else {
    const float pmax2 = fmaxf(px2, py2), pmin2 = fminf(px2, py2);
    int n = f.max_aniso;
    for (int i = 1; i < f.max_aniso; ++i)
      if (__fmul_rn((float)(i * i), pmin2) >= pmax2) {
        n = i;
        break;
      }
    b.lod = 0.5f * __log2f(pmax2) - __log2f((float)n);
    const bool major_x = px2 >= py2;
    b.n = n;
    b.du = major_x ? d.x : d.z;
    b.dv = major_x ? d.y : d.w;
    b.inv = 1.0f / (float)(n + 1);
  }
  return b;
}

// Level of detail of level k clamped to its mip range, from a base whose
// level of detail is `shift` above this level's (NaN and -inf give 0).
__device__ __forceinline__ float clamped_lod(const FilterArgs &f, int k, float lod, float shift) {
  return fminf(fmaxf(lod - shift, 0.0f), (float)(f.n_mips[k] - 1));
}

// Selection on level k from a base whose level of detail is `shift` above
// this level's.
__device__ __forceinline__ LodSel lod_select(const FilterArgs &f, int k, const LodBase &b, float shift) {
  LodSel s;
  const int nm = f.n_mips[k];
  const float lod = clamped_lod(f, k, b.lod, shift);
  int m0 = (int)floorf(lod);
  m0 = m0 < 0 ? 0 : (m0 > nm - 1 ? nm - 1 : m0);
  const float t = lod - (float)m0;
  s.m0 = m0;
  s.t = (t > 0.0f && m0 + 1 < nm) ? t : 0.0f;
  s.n = b.n;
  s.du = b.du;
  s.dv = b.dv;
  s.inv = b.inv;
  return s;
}

// The same selection when the base's level of detail is a non-negative
// integer e above this level's, from the floor fl and fraction fr of the
// base's (clamped to [-64, 64], NaN to -64): where the level's value
// lod - e is not clamped it is exact, so its floor is fl - e and its
// fraction fr; where it is, the first or the last mip is taken alone.
__device__ __forceinline__ LodSel lod_select_int(const FilterArgs &f, int k, const LodBase &b, int fl, float fr) {
  LodSel s;
  const int last = f.n_mips[k] - 1;
  const int m = fl - f.shift_i[k];
  s.m0 = min(max(m, 0), last);
  s.t = (unsigned)m < (unsigned)last ? fr : 0.0f;  // 0 <= m < last
  s.n = b.n;
  s.du = b.du;
  s.dv = b.dv;
  s.inv = b.inv;
  return s;
}

// Offset of anisotropic tap i (1..n) along the major axis, in units of it:
// i / (n + 1) - 1/2, with inv = 1 / (n + 1) (monotonic in i).
__device__ __forceinline__ float aniso_offset(int i, float inv) { return fmaf((float)i, inv, -0.5f); }

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
    const float t = aniso_offset(i, s.inv);
    const float3 c = tri(fmaf(t, s.du, u), fmaf(t, s.dv, v));
    acc.x += c.x;
    acc.y += c.y;
    acc.z += c.z;
  }
  const float inv = 1.0f / (float)s.n;
  return make_float3(acc.x * inv, acc.y * inv, acc.z * inv);
}

// Trilinear features of one level in packed FP16: the sample of mip m0,
// blended towards the sample of mip m0 + 1 by t (a subtraction and a fused
// multiply-add per channel pair; the constant 1 of the (b, 1) pair stays 1).
template <class SMP>
__device__ __forceinline__ Tex16 trilinear16(const LodSel &s, float u, float v, SMP &&smp) {
  Tex16 c = smp(s.m0, u, v);
  if (s.t > 0.0f) {
    const Tex16 c1 = smp(s.m0 + 1, u, v);
    const _Float16 th = (_Float16)s.t;
    const half2_t t2 = {th, th};
    c.rg = __builtin_elementwise_fma(t2, c1.rg - c.rg, c.rg);
    c.b1 = __builtin_elementwise_fma(t2, c1.b1 - c.b1, c.b1);
  }
  return c;
}

// Staged regions of one span: region r = 2 k + j is mip m_lo[k] + j of level
// k; bit r of `staged` is set when its texels are in LDS, texel (i, j) at
// kbase[r] + j kbw[r] + i.
struct FiltStage {
  int m_lo[kMaxLevels];
  unsigned staged;
  unsigned interior;  // bit r: every position of region r lies in [0, n - 2] on both axes
  int kbw[kRegions], kbase[kRegions];
};

// Wave-uniform footprint of a span: the extreme coordinates of every
// position of every used level, per level the lowest first mip m_lo and
// whether some sample reads mip m_lo + 1 (bit k of need_hi).
struct SpanFoot {
  float umin, umax, vmin, vmax;
  int m_lo[kMaxLevels];
  unsigned need_hi;
};

// Extreme coordinates of one pixel's positions: the pixel itself and, for
// anisotropic filtering, its first and last tap along the major axis (the
// taps are monotonic in i).
template <int FILTER>
__device__ __forceinline__ void extend_taps(const LodBase &b, float u, float v, float &umin, float &umax, float &vmin,
                                            float &vmax) {
  const float uc = tap_coord(u), vc = tap_coord(v);
  umin = fminf(umin, uc);
  umax = fmaxf(umax, uc);
  vmin = fminf(vmin, vc);
  vmax = fmaxf(vmax, vc);
  if (FILTER != 1) {
    const float ta = aniso_offset(1, b.inv), tb = aniso_offset(b.n, b.inv);
    const float xa = tap_coord(fmaf(ta, b.du, u)), xb = tap_coord(fmaf(tb, b.du, u));
    const float ya = tap_coord(fmaf(ta, b.dv, v)), yb = tap_coord(fmaf(tb, b.dv, v));
    umin = fminf(umin, fminf(xa, xb));
    umax = fmaxf(umax, fmaxf(xa, xb));
    vmin = fminf(vmin, fminf(ya, yb));
    vmax = fmaxf(vmax, fmaxf(ya, yb));
  }
}

// Mip range of level k over a span from the extremes of its clamped level
// of detail: floor and ceiling are monotonic, so the lowest first mip is the
// floor of the minimum and the highest mip read (m0, or m0 + 1 when t > 0)
// the ceiling of the maximum.
__device__ __forceinline__ void mip_range(const FilterArgs &f, int k, float lo, float hi, SpanFoot &ft) {
  const int nm = f.n_mips[k];
  int m = (int)floorf(lo);
  m = m < 0 ? 0 : (m > nm - 1 ? nm - 1 : m);
  ft.m_lo[k] = m;
  if ((int)ceilf(hi) > m) ft.need_hi |= 1u << k;
}

// Staging of the span's regions. stage: kFiltStageTexels texels; srec:
// 2 kRegions records. Regions are taken in order while they fit; a region of
// mip m_lo + 1 that no sample reads is left out.
__device__ __forceinline__ FiltStage stage_footprints(const FilterArgs &f, const SpanFoot &ft, uint2 *stage,
                                                      f32x4 *srec, int salt) {
  const int lane = threadIdx.x & 63;
  FiltStage st;
#pragma unroll
  for (int k = 0; k < kMaxLevels; ++k) st.m_lo[k] = ft.m_lo[k];
  // lane 4 r + q (r < kRegions): tap index of an extreme coordinate on
  // region r; q = 0: left tap of umin, 1: left tap of umax, 2: top tap of
  // vmin, 3: top tap of vmax
  const int r = (lane >> 2) & (kRegions - 1), q = lane & 3, k = r >> 1;
  const int mlo = k == 0 ? ft.m_lo[0] : (k == 1 ? ft.m_lo[1] : (k == 2 ? ft.m_lo[2] : ft.m_lo[3]));
  const int m = mlo + (r & 1);
  const bool valid = lane < 4 * kRegions && k < f.n_levels && m < f.n_mips[k] &&
                     ((r & 1) == 0 || ((ft.need_hi >> k) & 1u));
  const MipArgs &M = f.mip[k][valid ? m : 0];
  const bool ay = q >= 2;
  const float dim = ay ? M.fh : M.fw;
  const float ext = q == 0 ? ft.umin : (q == 1 ? ft.umax : (q == 2 ? ft.vmin : ft.vmax));
  const float cpos = (ay ? f.sy[k] : f.sx[k]) - 0.5f;
  const int ti = (int)tap_floor(ext, dim, cpos, dim - 2.0f);
  // the positions are monotonic in the coordinate: the extremes decide
  const float raw = fmaf(ext, dim, cpos);
  const unsigned long long outside =
      __builtin_amdgcn_ballot_w64(lane < 4 * kRegions && !(raw >= 0.0f && raw <= dim - 2.0f));
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
  st.interior = 0u;
#pragma unroll
  for (int rr = 0; rr < kRegions; ++rr)
    if (((outside >> (4 * rr)) & 0xFull) == 0) st.interior |= 1u << rr;
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
                                               int kbw, int kbase, float x, float y, bool interior) {
  int i0, j0;
  float fx, fy;
  if (interior) {
    // positions inside [0, n - 2]: floor and fraction as they stand, what
    // clamp_tap gives there
    const float px = fmaf(x, fw, cx), py = fmaf(y, fh, cy);
    i0 = (int)px;
    j0 = (int)py;
    fx = __builtin_amdgcn_fractf(px);
    fy = __builtin_amdgcn_fractf(py);
  } else {
    clamp_tap(tap_coord(x), fw, cx, fw - 2.0f, i0, fx);
    clamp_tap(tap_coord(y), fh, cy, fh - 2.0f, j0, fy);
  }
  const uint2 *t = stage + kbase + __mul24(j0, kbw) + i0;
  return lerp_tex16(tex16_from(t[0]), tex16_from(t[1]), tex16_from(t[kbw]), tex16_from(t[kbw + 1]), fx, fy);
}

// A span is SUBS sub-spans of 64 consecutive pixels: the footprints of all
// its pixels are staged once, then each sub-span is sampled and run through
// the MLP. Long spans spread the footprint reductions, the staging records
// and the partly filled staging passes over more pixels; trilinear spans
// take 1024 pixels, anisotropic ones (footprints stretched along the major
// axis) 256.
template <class P, int HID, int NL, int VEC4, int FILTER, int SUBS>
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
  constexpr int kSpanPx = 64 * SUBS;
  const int64_t n_span = (a.n + kSpanPx - 1) / kSpanPx;
  // shared level of detail with every level at or below level 0's size
  bool int_shift = f.shared_lod != 0;
#pragma unroll
  for (int k = 0; k < kMaxLevels; ++k)
    if (k < f.n_levels && f.lod_shift[k] < 0.0f) int_shift = false;
  // this lane's pixel of sub-span i of span s (pixels past the end repeat
  // the last one)
  auto pixel_of = [&](int64_t s, int i) {
    const int64_t p = s * kSpanPx + 64 * i + lane;
    return p < a.n ? p : a.n - 1;
  };
  // One-sub-span spans load their uv and derivatives one span ahead; longer
  // spans load theirs when they start (registers held through the MLP would
  // spill; the other wavefront of the SIMD works while the loads are in
  // flight).
  float2 uv_next = make_float2(0.f, 0.f);
  float4 d_next = make_float4(0.f, 0.f, 0.f, 0.f);
  if (SUBS == 1 && (int64_t)blockIdx.x < n_span) {
    const int64_t p = pixel_of(blockIdx.x, 0);
    uv_next = a.uv[p];
    d_next = f.duv[p];
  }
  for (int64_t s = blockIdx.x; s < n_span; s += gridDim.x) {
    float2 uv[SUBS];
    float4 d[SUBS];
    if constexpr (SUBS == 1) {
      uv[0] = uv_next;
      d[0] = d_next;
      if (s + gridDim.x < n_span) {
        const int64_t p = pixel_of(s + gridDim.x, 0);
        uv_next = a.uv[p];
        d_next = f.duv[p];
      }
    } else {
#pragma unroll
      for (int i = 0; i < SUBS; ++i) {
        const int64_t p = pixel_of(s, i);
        uv[i] = a.uv[p];
        d[i] = f.duv[p];
      }
    }
    // footprint of the span: per lane over its pixels, then over the wave
    float umin = __builtin_inff(), umax = -__builtin_inff(), vmin = __builtin_inff(), vmax = -__builtin_inff();
    SpanFoot ft;
    ft.need_hi = 0u;
    LodBase bs[SUBS];  // shared level of detail: the base of each pixel
    if (f.shared_lod) {
      // every level's clamped level of detail is monotonic in the base's
      float blo = __builtin_inff(), bhi = -__builtin_inff();
#pragma unroll
      for (int i = 0; i < SUBS; ++i) {
        bs[i] = lod_base<FILTER>(f, f.w0[0], f.h0[0], d[i]);
        const float l = fmaxf(bs[i].lod, -__builtin_inff());  // NaN as -inf: both clamp to 0
        blo = fminf(blo, l);
        bhi = fmaxf(bhi, l);
        extend_taps<FILTER>(bs[i], uv[i].x, uv[i].y, umin, umax, vmin, vmax);
      }
      blo = wave_min_key(blo);
      bhi = wave_max_key(bhi);
#pragma unroll
      for (int k = 0; k < kMaxLevels; ++k) {
        ft.m_lo[k] = 0;
        if (k < f.n_levels)
          mip_range(f, k, clamped_lod(f, k, blo, f.lod_shift[k]), clamped_lod(f, k, bhi, f.lod_shift[k]), ft);
      }
    } else {
      float lo[kMaxLevels], hi[kMaxLevels];
#pragma unroll
      for (int k = 0; k < kMaxLevels; ++k) {
        lo[k] = __builtin_inff();
        hi[k] = -__builtin_inff();
      }
#pragma unroll
      for (int i = 0; i < SUBS; ++i) {
#pragma unroll
        for (int k = 0; k < kMaxLevels; ++k) {
          const int kk = k < f.n_levels ? k : 0;
          const LodBase b = lod_base<FILTER>(f, f.w0[kk], f.h0[kk], d[i]);
          const float l = clamped_lod(f, kk, b.lod, 0.0f);
          lo[k] = fminf(lo[k], l);
          hi[k] = fmaxf(hi[k], l);
          extend_taps<FILTER>(b, uv[i].x, uv[i].y, umin, umax, vmin, vmax);
        }
      }
#pragma unroll
      for (int k = 0; k < kMaxLevels; ++k) {
        ft.m_lo[k] = 0;
        if (k < f.n_levels) mip_range(f, k, wave_min_key(lo[k]), wave_max_key(hi[k]), ft);
      }
    }
    ft.umin = wave_min_key(umin);
    ft.umax = wave_max_key(umax);
    ft.vmin = wave_min_key(vmin);
    ft.vmax = wave_max_key(vmax);
    // staged once for all the span's sub-spans (regions that do not fit are
    // fetched directly, which costs less than staging each sub-span on its
    // own)
    const FiltStage st = stage_footprints(f, ft, stage, srec, (int)s);
    // one sub-span per iteration (not unrolled: the code of a sub-span is
    // large). The uv and derivatives of sub-span i + 1 are loaded again
    // (from the cache) while sub-span i runs, so that no per-pixel array is
    // held through the MLP; the trilinear level of detail is recomputed, the
    // anisotropic base (with its tap count) moves to the front of bs.
    float2 uvc = uv[0];
    float4 dc = d[0];
#pragma unroll 1
    for (int i = 0; i < SUBS; ++i) {
      const int64_t first = s * kSpanPx + 64 * i;
      if (first >= a.n) break;
      const int64_t left = a.n - first;
      const float u = uvc.x, v = uvc.y;
      const float4 di = dc;
      if (SUBS > 1 && i + 1 < SUBS) {
        const int64_t p = pixel_of(s, i + 1);
        uvc = a.uv[p];
        dc = f.duv[p];
      }
      LodSel sel[kMaxLevels];
      if (f.shared_lod) {
        const LodBase b = FILTER == 1 ? lod_base<FILTER>(f, f.w0[0], f.h0[0], di) : bs[0];
        if (int_shift) {
          const float l = fminf(fmaxf(b.lod, -64.0f), 64.0f);
          const float fl = floorf(l);
          const float fr = l - fl;
#pragma unroll
          for (int k = 0; k < kMaxLevels; ++k)
            sel[k] = lod_select_int(f, k < f.n_levels ? k : 0, b, (int)fl, fr);
        } else {
#pragma unroll
          for (int k = 0; k < kMaxLevels; ++k) sel[k] = lod_select(f, k < f.n_levels ? k : 0, b, f.lod_shift[k]);
        }
      } else {
#pragma unroll
        for (int k = 0; k < kMaxLevels; ++k) {
          const int kk = k < f.n_levels ? k : 0;
          sel[k] = lod_select(f, kk, lod_base<FILTER>(f, f.w0[kk], f.h0[kk], di), 0.0f);
        }
      }
      if constexpr (FILTER != 1) {
#pragma unroll
        for (int j = 0; j + 1 < SUBS; ++j) bs[j] = bs[j + 1];
      }
      typename P::Frag bx[2];
      Tex16 c16[kMaxLevels];
      float xl[8], xh[8];
#pragma unroll
      for (int k = 0; k < kMaxLevels; ++k) {
        // levels past n_levels: zero features (their (b, 1) pads keep the
        // constant 1 of the bias slots)
        const half2_t z = {(_Float16)0.0f, (_Float16)0.0f}, z1 = {(_Float16)0.0f, (_Float16)1.0f};
        c16[k].rg = z;
        c16[k].b1 = z1;
        float3 c = make_float3(0.f, 0.f, 0.f);
        if (k < f.n_levels) {
          // this level's staged regions (the span's lowest mip m_lo and
          // m_lo + 1), as wave-uniform values
          const bool s0 = (st.staged >> (2 * k)) & 1u, s1 = (st.staged >> (2 * k + 1)) & 1u;
          const bool in0 = (st.interior >> (2 * k)) & 1u, in1 = (st.interior >> (2 * k + 1)) & 1u;
          const int mlo = __builtin_amdgcn_readfirstlane(st.m_lo[k]);
          // sizes of the two staged mips as wave-uniform values (a per-lane
          // choice between their addresses would load them per lane)
          const MipArgs &M0 = f.mip[k][mlo];
          const MipArgs &M1 = f.mip[k][mlo + 1 < kMaxMips ? mlo + 1 : mlo];
          const float fw0 = uniform_f(M0.fw), fh0 = uniform_f(M0.fh);
          const float fw1 = uniform_f(M1.fw), fh1 = uniform_f(M1.fh);
          const float cx = f.sx[k] - 0.5f, cy = f.sy[k] - 0.5f;
          const int kbw0 = st.kbw[2 * k], kbw1 = st.kbw[2 * k + 1];
          const int kb0 = st.kbase[2 * k], kb1 = st.kbase[2 * k + 1];
          // sample of mip m at (x, y): from a staged region or fetched directly
          auto smp = [&](int m, float x, float y) -> Tex16 {
            const int j = m - mlo;
            if ((j == 0 && s0) || (j == 1 && s1)) {
              const bool one = j == 1;
              return staged_sample(stage, one ? fw1 : fw0, one ? fh1 : fh0, cx, cy, one ? kbw1 : kbw0,
                                   one ? kb1 : kb0, x, y, one ? in1 : in0);
            }
            return sample_direct16(mip_level(f, k, m), tap_coord(x), tap_coord(y), 0);
          };
          // every lane reads mip m_lo alone (blend weight 0) and it is
          // staged: the samples take the region's values as wave-uniform
          // parameters (the same values as smp gives them)
          const bool lo_only = s0 && __builtin_amdgcn_ballot_w64(sel[k].m0 != mlo || sel[k].t > 0.0f) == 0;
          auto smp_lo = [&](int, float x, float y) -> Tex16 {
            return staged_sample(stage, fw0, fh0, cx, cy, kbw0, kb0, x, y, in0);
          };
          if constexpr (FILTER == 1) {
            if (lo_only)
              c16[k] = smp_lo(mlo, u, v);
            else
              c16[k] = trilinear16(sel[k], u, v, smp);
          } else {
            if (lo_only)
              c = filter_level<FILTER>(sel[k], u, v,
                                       [&](int m, float x, float y) { return tex_f3(smp_lo(m, x, y)); });
            else
              c = filter_level<FILTER>(sel[k], u, v, [&](int m, float x, float y) { return tex_f3(smp(m, x, y)); });
          }
        }
        if constexpr (FILTER != 1) put_level(xl, xh, k, c);
      }
      if constexpr (FILTER == 1) {
        // trilinear: FP16 samples blended in packed FP16 straight into the
        // first layer's operands
        operands16(c16, u, v, bx);
      } else {
        pixel_operands<P>(xl, xh, u, v, W.in_scale, bx);
      }
      const int span = left < 64 ? (int)left : 64;
      // ReLU by the [0, 1] clamp of the conversion when the image is scaled
      // for it and every coordinate of the sub-span lies in the unit square
      // (the features are then blends of latent values in [0, 1], as in the
      // unfiltered decode)
      const bool in_unit = __builtin_amdgcn_ballot_w64(!(u >= 0.0f && u <= 1.0f && v >= 0.0f && v <= 1.0f)) == 0;
      if (in_unit && W.unit_relu != 0)
        subspan_mlp<P, HID, NL, VEC4, true>(a, W, bias, span_out(a, first, span), bx, 0, (int)first);
      else
        subspan_mlp<P, HID, NL, VEC4, false>(a, W, bias, span_out(a, first, span), bx, 0, (int)first);
    }
  }
}

template <int HID, int VEC4, int FILTER>
hipError_t launch_nl(const FilterArgs &f, int n_layers, int grid, hipStream_t st) {
  constexpr int S = FILTER == 1 ? NTC_FILT_TRI_SUBS : NTC_FILT_ANI_SUBS;
  const size_t lds = (size_t)(BiasLds<HID, 5>::kCount + 2 * kRegions) * sizeof(f32x4) + kFiltStageTexels * sizeof(uint2);
  switch (n_layers) {
    case 2: hipLaunchKernelGGL((decode_filtered_kernel<PrecF16, HID, 2, VEC4, FILTER, S>), dim3(grid), dim3(64), lds, st, f); break;
    case 3: hipLaunchKernelGGL((decode_filtered_kernel<PrecF16, HID, 3, VEC4, FILTER, S>), dim3(grid), dim3(64), lds, st, f); break;
    case 4: hipLaunchKernelGGL((decode_filtered_kernel<PrecF16, HID, 4, VEC4, FILTER, S>), dim3(grid), dim3(64), lds, st, f); break;
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
  const int64_t span_px = 64 * (f.filter == 1 ? NTC_FILT_TRI_SUBS : NTC_FILT_ANI_SUBS);
  const int64_t n_span = (f.d.n + span_px - 1) / span_px;
  if (grid > n_span) grid = n_span;
  if (grid < 1) grid = 1;
  switch (s.hid) {
    case 16: return launch_vec<16>(f, s.n_layers, (int)grid, st);
    case 32: return launch_vec<32>(f, s.n_layers, (int)grid, st);
    case 64: return launch_vec<64>(f, s.n_layers, (int)grid, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ntc
