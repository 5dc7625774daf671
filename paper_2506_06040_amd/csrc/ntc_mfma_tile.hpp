// Matrix-core tile decode shared by the single-material and the batched
// kernels (see ntc_mfma.hip for the data layout).
//
// Per 64-pixel tile and wavefront (lane l = 16 g + n, lane group g samples
// latent level g for pixels 16 t + n, t = 0..3):
//   1. uv of the four pixels; the tile's uv extremes by DPP row reductions
//      (every lane group holds all 64 pixels, so every row reduces the whole
//      tile).
//   2. Bounding box of the taps on each level, from the uv extremes (the tap
//      position is monotone in uv). If the boxes fit the wave's LDS region,
//      every texel of them is decoded once (integer BC1 decode, then the
//      exact numerators scaled to FP32) into LDS, one level after another.
//   3. Bilinear taps read four adjacent texels from LDS. Clamp-to-edge is
//      applied to the sampling position instead of the taps: x is limited to
//      [0, w - 1] and the left tap to [0, w - 2], so the right tap is always
//      the next texel and an edge sample gets weight 1 on the edge texel.
//      This gives the same value as clamping both taps.
//   4. MLP on the matrix cores in two passes of 32 pixels; ReLU on packed
//      FP16 after conversion; sigmoid with the hardware exp2 / reciprocal.
#pragma once

#include <hip/hip_runtime.h>

#include "ntc_device.hpp"
#include "ntc_internal.hpp"

namespace ntc {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

#define NTC_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ T gload(const T *p) {
  return *(const NTC_GLOBAL T *)(p);
}
__device__ __forceinline__ uint2 gload2u(const uint2 *p) {
  const unsigned long long v = gload(reinterpret_cast<const unsigned long long *>(p));
  return make_uint2((unsigned)v, (unsigned)(v >> 32));
}
__device__ __forceinline__ float2 gload2f(const float2 *p) {
  const unsigned long long v = gload(reinterpret_cast<const unsigned long long *>(p));
  return make_float2(__uint_as_float((unsigned)v), __uint_as_float((unsigned)(v >> 32)));
}

__device__ __forceinline__ half2_t relu_pk(float a, float b) {
  const f32x2 v = {a, b};
  const half2_t h = __builtin_convertvector(v, half2_t);
  const half2_t z = {(_Float16)0.0f, (_Float16)0.0f};
  return __builtin_elementwise_max(h, z);
}

struct PrecF16 {
  using Frag = half8_t;
  static constexpr bool kScaled = false;
  __device__ __forceinline__ static f32x4 mma(Frag a, Frag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static Frag features(float r, float g, float b, float u, float v, float) {
    const f32x2 p0 = {r, g}, p1 = {b, u}, p2 = {v, 0.0f};
    const half2_t h0 = __builtin_convertvector(p0, half2_t);
    const half2_t h1 = __builtin_convertvector(p1, half2_t);
    const half2_t h2 = __builtin_convertvector(p2, half2_t);
    Frag f;
    f[0] = h0[0];
    f[1] = h0[1];
    f[2] = h1[0];
    f[3] = h1[1];
    f[4] = h2[0];
    f[5] = h2[1];
    f[6] = (_Float16)0.0f;
    f[7] = (_Float16)0.0f;
    return f;
  }
  __device__ __forceinline__ static Frag hidden(f32x4 lo, f32x4 hi, float) {
    const half2_t a = relu_pk(lo[0], lo[1]), b = relu_pk(lo[2], lo[3]);
    const half2_t c = relu_pk(hi[0], hi[1]), d = relu_pk(hi[2], hi[3]);
    Frag f;
    f[0] = a[0];
    f[1] = a[1];
    f[2] = b[0];
    f[3] = b[1];
    f[4] = c[0];
    f[5] = c[1];
    f[6] = d[0];
    f[7] = d[1];
    return f;
  }
};

// OCP E4M3 with saturation to +-448 (the conversion instruction is applied
// to clamped values).
__device__ __forceinline__ float sat448(float v) { return __builtin_amdgcn_fmed3f(v, -448.0f, 448.0f); }

__device__ __forceinline__ long pack_e4m3(float v0, float v1, float v2, float v3, float v4, float v5, float v6,
                                          float v7) {
  int lo = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(v0), sat448(v1), 0, false);
  lo = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(v2), sat448(v3), lo, true);
  int hi = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(v4), sat448(v5), 0, false);
  hi = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(v6), sat448(v7), hi, true);
  return (long)(((unsigned long)(unsigned)hi << 32) | (unsigned)lo);
}

struct PrecF8 {
  using Frag = long;
  static constexpr bool kScaled = true;
  __device__ __forceinline__ static f32x4 mma(Frag a, Frag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static Frag features(float r, float g, float b, float u, float v, float s) {
    return pack_e4m3(r * s, g * s, b * s, u * s, v * s, 0.f, 0.f, 0.f);
  }
  __device__ __forceinline__ static Frag hidden(f32x4 lo, f32x4 hi, float s) {
    return pack_e4m3(fmaxf(lo[0], 0.f) * s, fmaxf(lo[1], 0.f) * s, fmaxf(lo[2], 0.f) * s,
                     fmaxf(lo[3], 0.f) * s, fmaxf(hi[0], 0.f) * s, fmaxf(hi[1], 0.f) * s,
                     fmaxf(hi[2], 0.f) * s, fmaxf(hi[3], 0.f) * s);
  }
};

// Minimum / maximum over the 16 lanes of a DPP row (row rotations).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row_min(float v) {
  v = fminf(v, dpp_f<0x128>(v));
  v = fminf(v, dpp_f<0x124>(v));
  v = fminf(v, dpp_f<0x122>(v));
  v = fminf(v, dpp_f<0x121>(v));
  return v;
}
__device__ __forceinline__ float row_max(float v) {
  v = fmaxf(v, dpp_f<0x128>(v));
  v = fmaxf(v, dpp_f<0x124>(v));
  v = fmaxf(v, dpp_f<0x122>(v));
  v = fmaxf(v, dpp_f<0x121>(v));
  return v;
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ int row_min_i(int v) {
  v = min(v, dpp_i<0x128>(v));
  v = min(v, dpp_i<0x124>(v));
  v = min(v, dpp_i<0x122>(v));
  v = min(v, dpp_i<0x121>(v));
  return v;
}
__device__ __forceinline__ int row_max_i(int v) {
  v = max(v, dpp_i<0x128>(v));
  v = max(v, dpp_i<0x124>(v));
  v = max(v, dpp_i<0x122>(v));
  v = max(v, dpp_i<0x121>(v));
  return v;
}

__device__ __forceinline__ float uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// Register-resident weights of one MLP.
template <class P, int HID, int NL>
struct MfmaWeights {
  static constexpr int MT = HID / 16;
  static constexpr int KC = HID >= 32 ? HID / 32 : 1;
  static constexpr int NH = NL > 2 ? NL - 2 : 1;
  using Frag = typename P::Frag;
  Frag w0[MT];
  Frag wh[NH][MT][KC];
  Frag wo[KC];
  float epi[kMaxLayers];
  float in_scale;

  __device__ __forceinline__ void load(const uint8_t *packed, const PackLayout &lay, int lane) {
    const Frag *f = reinterpret_cast<const Frag *>(packed + lay.w_off[0]);
#pragma unroll
    for (int m = 0; m < MT; ++m) w0[m] = gload(f + m * 64 + lane);
#pragma unroll
    for (int h = 0; h < NL - 2; ++h) {
      const Frag *fh = reinterpret_cast<const Frag *>(packed + lay.w_off[1 + h]);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < KC; ++c) wh[h][m][c] = gload(fh + (m * KC + c) * 64 + lane);
    }
    const Frag *fo = reinterpret_cast<const Frag *>(packed + lay.w_off[NL - 1]);
#pragma unroll
    for (int c = 0; c < KC; ++c) wo[c] = gload(fo + c * 64 + lane);
    in_scale = 1.0f;
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) epi[l] = 1.0f;
    if (P::kScaled) {
      const float *sc = reinterpret_cast<const float *>(packed + lay.scale_off);
      in_scale = gload(sc);
#pragma unroll
      for (int l = 0; l < NL; ++l) epi[l] = gload(sc + 3 * l + 1);
    }
  }
};

// Per-lane view of the latent level sampled by its lane group.
struct LaneLevel {
  const uint2 *bc1;
  int w, h, bw;
  float fw, fh, sx, sy;
};

// Uniform copies of kernel-argument fields: selecting between these values
// (instead of between the argument's fields) keeps the compiler from
// turning the per-lane choice into a pointer into the argument block, which
// would force a private copy of the whole argument struct.
__device__ __forceinline__ int ufld(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float ufld(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ const uint2 *ufld(const uint2 *p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (const uint2 *)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ LaneLevel lane_level(const LatArgs &lat, int g) {
  LaneLevel r;
#define NTC_PICK(f)                                                                                     \
  ([&] {                                                                                                \
    const auto v0 = ufld(lat.lv[0].f), v1 = ufld(lat.lv[1].f), v2 = ufld(lat.lv[2].f),                 \
               v3 = ufld(lat.lv[3].f);                                                                   \
    return g == 0 ? v0 : (g == 1 ? v1 : (g == 2 ? v2 : v3));                                            \
  }())
  r.bc1 = NTC_PICK(bc1);
  r.w = NTC_PICK(w);
  r.h = NTC_PICK(h);
  r.bw = NTC_PICK(bw);
  r.fw = NTC_PICK(fw);
  r.fh = NTC_PICK(fh);
  r.sx = NTC_PICK(sx);
  r.sy = NTC_PICK(sy);
#undef NTC_PICK
  return r;
}

// Left/top tap index and fraction along one axis, clamp-to-edge: the index
// is clamped in the integer domain to [0, n - 2] (any input, NaN and
// infinities included, lands inside the level), the fraction to [0, 1], so
// an edge sample puts weight 1 on the edge texel.
__device__ __forceinline__ void clamp_tap(float u, float fw, float s, int cap, int &i0, float &fr) {
  const float x = fmaf(u, fw, -0.5f) + s;
  const int xi = (int)floorf(x);
  i0 = min(max(xi, 0), cap);
  fr = __builtin_amdgcn_fmed3f(x - (float)i0, 0.0f, 1.0f);
}

// Texel of a BC1 level as three FP32 channel values.
__device__ __forceinline__ float3 texel_f32(uint32_t p) {
  return make_float3(numer_r(p) * kInvDenRB, numer_g(p) * kInvDenG, numer_b(p) * kInvDenRB);
}

__device__ __forceinline__ float3 blend4(float3 t00, float3 t10, float3 t01, float3 t11, float fx, float fy) {
  const float gx = 1.0f - fx, gy = 1.0f - fy;
  const float w00 = gx * gy, w10 = fx * gy, w01 = gx * fy, w11 = fx * fy;
  float3 c;
  c.x = fmaf(w11, t11.x, fmaf(w01, t01.x, fmaf(w10, t10.x, w00 * t00.x)));
  c.y = fmaf(w11, t11.y, fmaf(w01, t01.y, fmaf(w10, t10.y, w00 * t00.y)));
  c.z = fmaf(w11, t11.z, fmaf(w01, t01.z, fmaf(w10, t10.z, w00 * t00.z)));
  return c;
}

__device__ __forceinline__ float3 texel_direct(const uint2 *bc1, int bw, int i, int j) {
  const uint2 blk = gload2u(bc1 + (int64_t)(j >> 2) * bw + (i >> 2));
  return texel_f32(bc1_numer(blk.x, blk.y, (uint32_t)(((j & 3) << 2) | (i & 3))));
}

// Sample of one level with direct block fetches; `mode` 0 clamp, 1 wrap.
__device__ __forceinline__ float3 sample_direct(const LaneLevel &L, float u, float v, int mode) {
  if (mode == 0) {
    int i0, j0;
    float fx, fy;
    clamp_tap(u, L.fw, L.sx, L.w - 2, i0, fx);
    clamp_tap(v, L.fh, L.sy, L.h - 2, j0, fy);
    return blend4(texel_direct(L.bc1, L.bw, i0, j0), texel_direct(L.bc1, L.bw, i0 + 1, j0),
                  texel_direct(L.bc1, L.bw, i0, j0 + 1), texel_direct(L.bc1, L.bw, i0 + 1, j0 + 1), fx, fy);
  }
  float x = fmaf(u, L.fw, -0.5f) + L.sx;
  float y = fmaf(v, L.fh, -0.5f) + L.sy;
  x = fminf(fmaxf(x, -16777216.0f), 16777216.0f);
  y = fminf(fmaxf(y, -16777216.0f), 16777216.0f);
  const float xf = floorf(x), yf = floorf(y);
  const int ix = (int)xf, iy = (int)yf;
  const int i0 = address_coord(ix, L.w, 1), i1 = address_coord(ix + 1, L.w, 1);
  const int j0 = address_coord(iy, L.h, 1), j1 = address_coord(iy + 1, L.h, 1);
  return blend4(texel_direct(L.bc1, L.bw, i0, j0), texel_direct(L.bc1, L.bw, i1, j0),
                texel_direct(L.bc1, L.bw, i0, j1), texel_direct(L.bc1, L.bw, i1, j1), x - xf, y - yf);
}

// Sigmoid on the hardware exp2 / reciprocal.
__device__ __forceinline__ float sigmoid_fast(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// ---------------------------------------------------------------------------
// Buffer resources: SGPR base + 32-bit offsets; accesses at or beyond
// num_records bytes read 0 / are dropped by the hardware.
// ---------------------------------------------------------------------------
constexpr int kBufferFlags = 0x00020000;  // gfx9-family raw buffer word 3

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufferFlags);
}

// MLP over two N-tiles (32 pixels: N-tiles t0, t0 + 1 of the iteration) and store.
template <class P, int HID, int NL>
__device__ __forceinline__ void mlp_store2(const DecodeArgs &a, const MfmaWeights<P, HID, NL> &W,
                                           __amdgpu_buffer_rsrc_t wrs, __amdgpu_buffer_rsrc_t ors,
                                           const typename P::Frag (&bx)[2], int t0) {
  constexpr int MT = HID / 16;
  constexpr int KC = HID >= 32 ? HID / 32 : 1;
  constexpr int NH = NL - 2;
  constexpr int NT = 2;
  using Frag = typename P::Frag;
  const int lane = threadIdx.x;
  const int g = lane >> 4;
  const int nl = lane & 15;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};

  f32x4 acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const f32x4 bm = __builtin_bit_cast(
        f32x4, __builtin_amdgcn_raw_buffer_load_b128(wrs, g * 16, (int)a.lay.b_off[0] + m * 64, 0));
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = P::mma(W.w0[m], bx[t], bm);
  }
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    Frag hb[KC][NT];
#pragma unroll
    for (int c = 0; c < KC; ++c)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        hb[c][t] = P::hidden(acc[2 * c][t], (2 * c + 1 < MT) ? acc[(2 * c + 1) % MT][t] : zero, W.epi[h]);
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const f32x4 bm = __builtin_bit_cast(
          f32x4, __builtin_amdgcn_raw_buffer_load_b128(wrs, g * 16, (int)a.lay.b_off[1 + h] + m * 64, 0));
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        f32x4 s = P::mma(W.wh[h][m][0], hb[0][t], bm);
#pragma unroll
        for (int c = 1; c < KC; ++c) s = P::mma(W.wh[h][m][c], hb[c][t], s);
        acc[m][t] = s;
      }
    }
  }
  Frag hb[KC][NT];
#pragma unroll
  for (int c = 0; c < KC; ++c)
#pragma unroll
    for (int t = 0; t < NT; ++t)
      hb[c][t] = P::hidden(acc[2 * c][t], (2 * c + 1 < MT) ? acc[(2 * c + 1) % MT][t] : zero, W.epi[NL - 2]);
  const f32x4 bo = __builtin_bit_cast(
      f32x4, __builtin_amdgcn_raw_buffer_load_b128(wrs, g * 16, (int)a.lay.b_off[NL - 1], 0));
  const float out_scale = P::kScaled ? W.epi[NL - 1] : 1.0f;
  const int n_out = a.n_out;
  const int esz = a.out_f16 ? 2 : 4;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    f32x4 z = P::mma(W.wo[0], hb[0][t], bo);
#pragma unroll
    for (int c = 1; c < KC; ++c) z = P::mma(W.wo[c], hb[c][t], z);
    if (4 * g < n_out) {
      f32x4 f;
#pragma unroll
      for (int i = 0; i < 4; ++i) f[i] = sigmoid_fast(P::kScaled ? z[i] * out_scale : z[i]);
      // pixels past the end of the batch fall outside the buffer and are dropped
      const int off = ((16 * (t0 + t) + nl) * n_out + 4 * g) * esz;
      if ((n_out & 3) == 0) {
        if (a.out_f16) {
          const half4_t hv = __builtin_convertvector(f, half4_t);
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, hv),
                                                ors, off, 0, 2);
        } else {
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, f),
                                                 ors, off, 0, 2);
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (4 * g + i < n_out) {
            // element copied to a scalar first: bit-casting a vector element
            // in place reads element 0 with this compiler
            const float fi = f[i];
            if (a.out_f16) {
              const _Float16 hi = (_Float16)fi;
              __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, hi), ors, off + 2 * i, 0, 2);
            } else {
              __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(fi), ors, off + 4 * i, 0, 2);
            }
          }
        }
      }
    }
  }
}

// Decode TP consecutive 64-pixel tiles starting at tile `tile`: stage, sample,
// run the MLP, store. Lane (g, n) owns pixels 16 t + n, t < 4 TP, of the
// 64 TP-pixel span. stage: this wave's LDS region of a.stage_cap texels.
// end_px bounds the pixels this call may write (the batch end, or the end
// of a work item).
template <class P, int HID, int NL, int TP>
__device__ __forceinline__ void decode_tiles(const DecodeArgs &a, const LaneLevel &L, bool has_level, int64_t tile,
                                             int64_t end_px, f32x4 *stage, const MfmaWeights<P, HID, NL> &W,
                                             __amdgpu_buffer_rsrc_t wrs) {
  using Frag = typename P::Frag;
  constexpr int NP = 4 * TP;  // pixels per lane
  const int lane = threadIdx.x;
  const int g = lane >> 4;
  const int nl = lane & 15;
  const int mode = a.lat.address;

  const int64_t base = tile * 64;
  const int64_t left = end_px - base;
  const int span = left < 64 * TP ? (int)left : 64 * TP;
  const int esz = a.out_f16 ? 2 : 4;
  const __amdgpu_buffer_rsrc_t urs = make_rsrc(a.uv + base, (uint32_t)span * 8u);
  const __amdgpu_buffer_rsrc_t ors =
      make_rsrc(reinterpret_cast<const char *>(a.out) + base * a.n_out * esz, (uint32_t)(span * a.n_out * esz));

  float u[NP], v[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    const auto q = __builtin_amdgcn_raw_buffer_load_b64(urs, nl * 8, t * 128, 0);
    u[t] = __uint_as_float(q[0]);
    v[t] = __uint_as_float(q[1]);
  }

  float3 c[NP];
  bool staged = false;
  if (mode == 0) {
    // taps of this lane group's level; the row reduction of the left/top
    // taps gives the level's box (left taps in [bx, bx + bw - 2])
    int ti[NP], tj[NP];
    float fx[NP], fy[NP];
    int x0 = 0x7fffffff, x1 = -1, y0 = 0x7fffffff, y1 = -1;
#pragma unroll
    for (int t = 0; t < NP; ++t) {
      clamp_tap(u[t], L.fw, L.sx, L.w - 2, ti[t], fx[t]);
      clamp_tap(v[t], L.fh, L.sy, L.h - 2, tj[t], fy[t]);
      x0 = min(x0, ti[t]);
      x1 = max(x1, ti[t]);
      y0 = min(y0, tj[t]);
      y1 = max(y1, tj[t]);
    }
    x0 = row_min_i(x0);
    x1 = row_max_i(x1);
    y0 = row_min_i(y0);
    y1 = row_max_i(y1);
    const int bw = has_level ? x1 - x0 + 2 : 0;
    const int bh = has_level ? y1 - y0 + 2 : 0;
    const int cnt = bw * bh;
    const int c0 = __builtin_amdgcn_readlane(cnt, 0), c1 = __builtin_amdgcn_readlane(cnt, 16);
    const int c2 = __builtin_amdgcn_readlane(cnt, 32), c3 = __builtin_amdgcn_readlane(cnt, 48);
    if (c0 + c1 + c2 + c3 <= a.stage_cap) {
      staged = true;
      const int cnts[4] = {c0, c1, c2, c3};
      int gbase = 0, my_base = 0;
#pragma unroll
      for (int k = 0; k < kMaxLevels; ++k) {
        if (g == k) my_base = gbase;
        const int ck = cnts[k];
        if (ck > 0) {
          const LevelArgs &Lk = a.lat.lv[k];
          const __amdgpu_buffer_rsrc_t brs = make_rsrc(Lk.bc1, (uint32_t)(Lk.bw * (Lk.h >> 2)) * 8u);
          const int kbx = __builtin_amdgcn_readlane(x0, 16 * k);
          const int kby = __builtin_amdgcn_readlane(y0, 16 * k);
          const int kbw = __builtin_amdgcn_readlane(bw, 16 * k);
          const float rcp = __builtin_amdgcn_rcpf((float)kbw);
          for (int t = lane; t < ck; t += 64) {
            // exact: (t + 1/2) / bw is at least 1/(2 bw) from an integer and the
            // reciprocal's relative error (~2^-22) moves it by < 1e-3 / bw
            const int ty = (int)(((float)t + 0.5f) * rcp);
            const int tx = t - ty * kbw;
            const int X = kbx + tx, Y = kby + ty;
            const auto blk = __builtin_amdgcn_raw_buffer_load_b64(brs, ((Y >> 2) * Lk.bw + (X >> 2)) * 8, 0, 0);
            const float3 val = texel_f32(bc1_numer(blk[0], blk[1], (uint32_t)(((Y & 3) << 2) | (X & 3))));
            const f32x4 s4 = {val.x, val.y, val.z, 0.0f};
            stage[gbase + t] = s4;
          }
        }
        gbase += ck;
      }
      __syncthreads();
      if (has_level) {
#pragma unroll
        for (int t = 0; t < NP; ++t) {
          const int r = my_base + (tj[t] - y0) * bw + (ti[t] - x0);
          const f32x4 t00 = stage[r], t10 = stage[r + 1], t01 = stage[r + bw], t11 = stage[r + bw + 1];
          c[t] = blend4(make_float3(t00[0], t00[1], t00[2]), make_float3(t10[0], t10[1], t10[2]),
                        make_float3(t01[0], t01[1], t01[2]), make_float3(t11[0], t11[1], t11[2]), fx[t], fy[t]);
        }
      }
      __syncthreads();
    }
  }
  if (!staged && has_level) {
#pragma unroll
    for (int t = 0; t < NP; ++t) c[t] = sample_direct(L, u[t], v[t], mode);
  }

#pragma unroll
  for (int p = 0; p < 2 * TP; ++p) {
    Frag bx[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int t = 2 * p + q;
      const float3 cc = has_level ? c[t] : make_float3(0.f, 0.f, 0.f);
      bx[q] = P::features(cc.x, cc.y, cc.z, g == 0 ? u[t] : 0.f, g == 0 ? v[t] : 0.f, W.in_scale);
    }
    mlp_store2<P, HID, NL>(a, W, wrs, ors, bx, 2 * p);
  }
}

}  // namespace ntc
