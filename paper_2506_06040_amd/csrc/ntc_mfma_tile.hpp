// Matrix-core tile decode shared by the single-material and the batched
// kernels (see ntc_mfma.hip for the data layout).
#pragma once

#include <hip/hip_runtime.h>

#include "ntc_device.hpp"
#include "ntc_internal.hpp"

namespace ntc {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

struct PrecF16 {
  using Frag = half8_t;
  static constexpr bool kScaled = false;
  __device__ __forceinline__ static f32x4 mma(Frag a, Frag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static Frag features(float r, float g, float b, float u, float v, float) {
    Frag f;
    f[0] = (_Float16)r;
    f[1] = (_Float16)g;
    f[2] = (_Float16)b;
    f[3] = (_Float16)u;
    f[4] = (_Float16)v;
    f[5] = (_Float16)0.0f;
    f[6] = (_Float16)0.0f;
    f[7] = (_Float16)0.0f;
    return f;
  }
  __device__ __forceinline__ static Frag hidden(f32x4 lo, f32x4 hi, float) {
    Frag f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f[i] = (_Float16)fmaxf(lo[i], 0.0f);
      f[4 + i] = (_Float16)fmaxf(hi[i], 0.0f);
    }
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

__device__ __forceinline__ int group_min(int v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 16));
  return v;
}
__device__ __forceinline__ int group_max(int v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 16));
  return v;
}

template <class T>
__device__ __forceinline__ T pick4(int k, T a0, T a1, T a2, T a3) {
  return k == 0 ? a0 : (k == 1 ? a1 : (k == 2 ? a2 : a3));
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
    for (int m = 0; m < MT; ++m) w0[m] = f[m * 64 + lane];
#pragma unroll
    for (int h = 0; h < NL - 2; ++h) {
      const Frag *fh = reinterpret_cast<const Frag *>(packed + lay.w_off[1 + h]);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < KC; ++c) wh[h][m][c] = fh[(m * KC + c) * 64 + lane];
    }
    const Frag *fo = reinterpret_cast<const Frag *>(packed + lay.w_off[NL - 1]);
#pragma unroll
    for (int c = 0; c < KC; ++c) wo[c] = fo[c * 64 + lane];
    in_scale = 1.0f;
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) epi[l] = 1.0f;
    if (P::kScaled) {
      const float *sc = reinterpret_cast<const float *>(packed + lay.scale_off);
      in_scale = sc[0];
#pragma unroll
      for (int l = 0; l < NL; ++l) epi[l] = sc[3 * l + 1];
    }
  }
};

// Per-lane-group latent level.
__device__ __forceinline__ LevelArgs select_level(const LatArgs &lat, int g) {
  LevelArgs L = lat.lv[0];
  if (g == 1) L = lat.lv[1];
  if (g == 2) L = lat.lv[2];
  if (g == 3) L = lat.lv[3];
  return L;
}

// Decode one 64-pixel tile: stage, sample, run the MLP, store.
template <class P, int HID, int NL>
__device__ __forceinline__ void decode_tile(const DecodeArgs &a, const LevelArgs &L, bool has_level, int64_t tile,
                                            uint32_t *stage, const MfmaWeights<P, HID, NL> &W) {
  constexpr int MT = HID / 16;
  constexpr int KC = HID >= 32 ? HID / 32 : 1;
  constexpr int NH = NL - 2;
  using Frag = typename P::Frag;
  const int lane = threadIdx.x;
  const int g = lane >> 4;
  const int nl = lane & 15;
  const int mode = a.lat.address;

  const int64_t base = tile * 64;
  float u[4], v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    int64_t p = base + 16 * t + nl;
    if (p >= a.n) p = a.n - 1;
    const float2 q = a.uv[p];
    u[t] = q.x;
    v[t] = q.y;
  }

  // Footprint of the tile on this lane group's level.
  Taps tp[4];
  int xmin = 0x7fffffff, xmax = -1, ymin = 0x7fffffff, ymax = -1;
  if (has_level) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      tp[t] = tap_coords(u[t], v[t], L, mode);
      xmin = min(xmin, min(tp[t].i0, tp[t].i1));
      xmax = max(xmax, max(tp[t].i0, tp[t].i1));
      ymin = min(ymin, min(tp[t].j0, tp[t].j1));
      ymax = max(ymax, max(tp[t].j0, tp[t].j1));
    }
  }
  xmin = group_min(xmin);
  ymin = group_min(ymin);
  xmax = group_max(xmax);
  ymax = group_max(ymax);
  const int bwid = has_level ? xmax - xmin + 1 : 0;
  const int cnt = has_level ? bwid * (ymax - ymin + 1) : 0;
  const int c0 = __builtin_amdgcn_readlane(cnt, 0), c1 = __builtin_amdgcn_readlane(cnt, 16);
  const int c2 = __builtin_amdgcn_readlane(cnt, 32), c3 = __builtin_amdgcn_readlane(cnt, 48);
  const int total = c0 + c1 + c2 + c3;

  uint32_t w00[4], w10[4], w01[4], w11[4];
  if (total <= a.stage_cap) {
    const int b1 = c0, b2 = c0 + c1, b3 = c0 + c1 + c2;
    const int x0_0 = __builtin_amdgcn_readlane(xmin, 0), x0_1 = __builtin_amdgcn_readlane(xmin, 16);
    const int x0_2 = __builtin_amdgcn_readlane(xmin, 32), x0_3 = __builtin_amdgcn_readlane(xmin, 48);
    const int y0_0 = __builtin_amdgcn_readlane(ymin, 0), y0_1 = __builtin_amdgcn_readlane(ymin, 16);
    const int y0_2 = __builtin_amdgcn_readlane(ymin, 32), y0_3 = __builtin_amdgcn_readlane(ymin, 48);
    const int bw_0 = __builtin_amdgcn_readlane(bwid, 0), bw_1 = __builtin_amdgcn_readlane(bwid, 16);
    const int bw_2 = __builtin_amdgcn_readlane(bwid, 32), bw_3 = __builtin_amdgcn_readlane(bwid, 48);
    // Every texel of the four boxes is decoded once into LDS.
    for (int t = lane; t < total; t += 64) {
      const int gg = (t >= b1) + (t >= b2) + (t >= b3);
      const int gb = pick4(gg, 0, b1, b2, b3);
      const int bx = pick4(gg, x0_0, x0_1, x0_2, x0_3);
      const int by = pick4(gg, y0_0, y0_1, y0_2, y0_3);
      const int bw = pick4(gg, bw_0, bw_1, bw_2, bw_3);
      const uint2 *blocks = pick4(gg, a.lat.lv[0].bc1, a.lat.lv[1].bc1, a.lat.lv[2].bc1, a.lat.lv[3].bc1);
      const int lw = pick4(gg, a.lat.lv[0].w, a.lat.lv[1].w, a.lat.lv[2].w, a.lat.lv[3].w);
      const int lh = pick4(gg, a.lat.lv[0].h, a.lat.lv[1].h, a.lat.lv[2].h, a.lat.lv[3].h);
      const int lbw = pick4(gg, a.lat.lv[0].bw, a.lat.lv[1].bw, a.lat.lv[2].bw, a.lat.lv[3].bw);
      const int r = t - gb;
      // exact: (r + 1/2) / bw is at least 1/(2 bw) away from an integer and
      // the reciprocal's relative error (~2^-22) keeps the product within
      // 1e-3 / bw of it for r < 4096
      const int ty = (int)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)bw));
      const int tx = r - ty * bw;
      const int X = min(max(bx + tx, 0), lw - 1);
      const int Y = min(max(by + ty, 0), lh - 1);
      const uint2 blk = blocks[(int64_t)(Y >> 2) * lbw + (X >> 2)];
      stage[t] = bc1_numer(blk.x, blk.y, (uint32_t)(((Y & 3) << 2) | (X & 3)));
    }
    __syncthreads();
    if (has_level) {
      const int gb = pick4(g, 0, b1, b2, b3);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r0 = gb + (tp[t].j0 - ymin) * bwid, r1 = gb + (tp[t].j1 - ymin) * bwid;
        w00[t] = stage[r0 + tp[t].i0 - xmin];
        w10[t] = stage[r0 + tp[t].i1 - xmin];
        w01[t] = stage[r1 + tp[t].i0 - xmin];
        w11[t] = stage[r1 + tp[t].i1 - xmin];
      }
    }
    __syncthreads();
  } else if (has_level) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      w00[t] = bc1_texel_global(L, tp[t].i0, tp[t].j0);
      w10[t] = bc1_texel_global(L, tp[t].i1, tp[t].j0);
      w01[t] = bc1_texel_global(L, tp[t].i0, tp[t].j1);
      w11[t] = bc1_texel_global(L, tp[t].i1, tp[t].j1);
    }
  }

  // Feature operand (layer 0 B operand).
  Frag bx[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float3 c = make_float3(0.f, 0.f, 0.f);
    if (has_level) c = blend_numer(w00[t], w10[t], w01[t], w11[t], tp[t].fx, tp[t].fy);
    const float uu = g == 0 ? u[t] : 0.f, vv = g == 0 ? v[t] : 0.f;
    bx[t] = P::features(c.x, c.y, c.z, uu, vv, W.in_scale);
  }

  const f32x4 *bias0 = reinterpret_cast<const f32x4 *>(a.packed + a.lay.b_off[0]);
  f32x4 acc[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const f32x4 bm = bias0[m * 4 + g];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[m][t] = P::mma(W.w0[m], bx[t], bm);
  }

#pragma unroll
  for (int h = 0; h < NH; ++h) {
    Frag hb[KC][4];
#pragma unroll
    for (int c = 0; c < KC; ++c)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
        hb[c][t] = P::hidden(acc[2 * c][t], (2 * c + 1 < MT) ? acc[(2 * c + 1) % MT][t] : zero, W.epi[h]);
      }
    const f32x4 *bias = reinterpret_cast<const f32x4 *>(a.packed + a.lay.b_off[1 + h]);
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const f32x4 bm = bias[m * 4 + g];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        f32x4 s = P::mma(W.wh[h][m][0], hb[0][t], bm);
#pragma unroll
        for (int c = 1; c < KC; ++c) s = P::mma(W.wh[h][m][c], hb[c][t], s);
        acc[m][t] = s;
      }
    }
  }

  Frag hb[KC][4];
#pragma unroll
  for (int c = 0; c < KC; ++c)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
      hb[c][t] = P::hidden(acc[2 * c][t], (2 * c + 1 < MT) ? acc[(2 * c + 1) % MT][t] : zero, W.epi[NL - 2]);
    }
  const f32x4 bo = reinterpret_cast<const f32x4 *>(a.packed + a.lay.b_off[NL - 1])[g];
  const float out_scale = P::kScaled ? W.epi[NL - 1] : 1.0f;
  const int n_out = a.n_out;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 z = P::mma(W.wo[0], hb[0][t], bo);
#pragma unroll
    for (int c = 1; c < KC; ++c) z = P::mma(W.wo[c], hb[c][t], z);
    const int64_t p = base + 16 * t + nl;
    if (p < a.n && 4 * g < n_out) {
      f32x4 f;
#pragma unroll
      for (int i = 0; i < 4; ++i) f[i] = __fdividef(1.0f, 1.0f + __expf(-z[i] * out_scale));
      if ((n_out & 3) == 0) {
        if (a.out_f16) {
          half4_t hv;
#pragma unroll
          for (int i = 0; i < 4; ++i) hv[i] = (_Float16)f[i];
          __builtin_nontemporal_store(hv, reinterpret_cast<half4_t *>(reinterpret_cast<_Float16 *>(a.out) +
                                                                       p * n_out + 4 * g));
        } else {
          __builtin_nontemporal_store(f, reinterpret_cast<f32x4 *>(reinterpret_cast<float *>(a.out) +
                                                                    p * n_out + 4 * g));
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (4 * g + i < n_out) {
            if (a.out_f16)
              reinterpret_cast<_Float16 *>(a.out)[p * n_out + 4 * g + i] = (_Float16)f[i];
            else
              reinterpret_cast<float *>(a.out)[p * n_out + 4 * g + i] = f[i];
          }
        }
      }
    }
  }
}

}  // namespace ntc
