// Device-side building blocks shared by the decode kernels of libntc.
//
// BC1 texel decode (Sec. 3.1, latent BC1 compression): a texel is
// (1 - a) e0 + a e1 with RGB565 endpoints per 4x4 block and a 2-bit index
// per texel, using the Khronos BC1 palette modes. Everything here is
// integer arithmetic: a texel becomes three exact numerators over the
// common denominator 6 (2^b - 1) (186 for the 5-bit red/blue channels, 378
// for the 6-bit green channel), packed into one 32-bit word
//     red | blue << 8 | green << 16.
// Bilinear sampling (Sec. 3.3) and the level shift (Sec. 3.1, variants)
// are in tap_coords().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ntc {

constexpr int kMaxLevels = 4;
constexpr int kMaxLayers = 5;
constexpr float kInvDenRB = 1.0f / 186.0f;
constexpr float kInvDenG = 1.0f / 378.0f;

struct LevelArgs {
  const uint2 *bc1;    // BC1 blocks: x = c0 | c1 << 16, y = index word
  const float *grid;   // float latents [h][w][3]
  int32_t w, h;        // texels
  int32_t bw;          // blocks per row (w / 4)
  int32_t pad_;
  float fw, fh;        // w, h as float
  float sx, sy;        // sampling offset in texels
};

struct LatArgs {
  LevelArgs lv[kMaxLevels];
  int32_t n_levels;
  int32_t format;      // 0 = BC1, 1 = float grids
  int32_t address;     // 0 = clamp, 1 = wrap
  int32_t pad_;
};

// A zero the compiler cannot see through, computed from a loop-variant
// (wavefront-uniform) `salt`. Offsetting a table pointer by it inside a loop
// keeps loop-invariant code motion from turning the table (bias fragments,
// level parameters, weights) into registers held across the loop, and keeps
// two reads of one value in different places from being merged; the table is
// read again where it is used instead. The asm is not volatile, so it orders
// no memory access and the scheduler stays free to interleave the reads.
__device__ __forceinline__ int opaque_zero(int salt) {
  int z;
  asm("s_mov_b32 %0, 0 ; %1" : "=s"(z) : "s"(salt));
  return z;
}

// Endpoint fields of an RGB565 word rearranged as red | blue << 8 | green << 16.
__device__ __forceinline__ uint32_t endpoint_fields(uint32_t c) {
  return (c >> 11) | ((c & 31u) << 8) | (((c >> 5) & 63u) << 16);
}

// Packed numerators of texel `pos` (= 4 y + x inside the block).
// Blend weights in sixths of (e0, e1) per index:
//   c0 > c1 : (6,0) (0,6) (4,2) (2,4)        -> e0, e1, (2e0+e1)/3, (e0+2e1)/3
//   c0 <= c1: (6,0) (0,6) (3,3) (0,0)        -> e0, e1, (e0+e1)/2, black
// The tables are stored as nibbles indexed by the 2-bit index. No field can
// carry into the next: 6 * 31 = 186 < 256 and 6 * 63 = 378 < 512.
__device__ __forceinline__ uint32_t bc1_numer(uint32_t lo, uint32_t hi, uint32_t pos) {
  const uint32_t c0 = lo & 0xFFFFu, c1 = lo >> 16;
  const uint32_t idx = (hi >> (2u * pos)) & 3u;
  const bool four = c0 > c1;
  const uint32_t t0 = four ? 0x2406u : 0x0306u;
  const uint32_t t1 = four ? 0x4260u : 0x0360u;
  const uint32_t a0 = (t0 >> (4u * idx)) & 15u;
  const uint32_t a1 = (t1 >> (4u * idx)) & 15u;
  return a0 * endpoint_fields(c0) + a1 * endpoint_fields(c1);
}

__device__ __forceinline__ float numer_r(uint32_t p) { return (float)(p & 255u); }
__device__ __forceinline__ float numer_b(uint32_t p) { return (float)((p >> 8) & 255u); }
__device__ __forceinline__ float numer_g(uint32_t p) { return (float)(p >> 16); }

// Texel word of level texel (i, j) fetched straight from the block array.
__device__ __forceinline__ uint32_t bc1_texel_global(const LevelArgs &L, int i, int j) {
  const uint2 blk = L.bc1[(int64_t)(j >> 2) * L.bw + (i >> 2)];
  return bc1_numer(blk.x, blk.y, (uint32_t)(((j & 3) << 2) | (i & 3)));
}

struct Taps {
  int i0, i1, j0, j1;  // tap columns / rows after addressing
  float fx, fy;        // bilinear fractions
};

__device__ __forceinline__ int address_coord(int i, int n, int mode) {
  if (mode == 1) {
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  return min(max(i, 0), n - 1);
}

// Bilinear footprint on one level: x = u w - 1/2 + s (texel centres at
// (i + 1/2) / w), taps floor(x) and floor(x) + 1, fraction x - floor(x).
// The position is first limited to +-2^24 texels so that every index stays
// inside the level whatever the input (NaN maps to -2^24).
__device__ __forceinline__ Taps tap_coords(float u, float v, const LevelArgs &L, int mode) {
  float x = fmaf(u, L.fw, -0.5f) + L.sx;
  float y = fmaf(v, L.fh, -0.5f) + L.sy;
  x = fminf(fmaxf(x, -16777216.0f), 16777216.0f);
  y = fminf(fmaxf(y, -16777216.0f), 16777216.0f);
  const float xf = floorf(x), yf = floorf(y);
  Taps t;
  t.fx = x - xf;
  t.fy = y - yf;
  const int ix = (int)xf, iy = (int)yf;
  t.i0 = address_coord(ix, L.w, mode);
  t.i1 = address_coord(ix + 1, L.w, mode);
  t.j0 = address_coord(iy, L.h, mode);
  t.j1 = address_coord(iy + 1, L.h, mode);
  return t;
}

// Bilinear blend of four packed BC1 texel words; returns the channel values.
__device__ __forceinline__ float3 blend_numer(uint32_t t00, uint32_t t10, uint32_t t01, uint32_t t11,
                                              float fx, float fy) {
  const float gx = 1.0f - fx, gy = 1.0f - fy;
  const float w00 = gx * gy, w10 = fx * gy, w01 = gx * fy, w11 = fx * fy;
  float r = w00 * numer_r(t00);
  r = fmaf(w10, numer_r(t10), r);
  r = fmaf(w01, numer_r(t01), r);
  r = fmaf(w11, numer_r(t11), r);
  float g = w00 * numer_g(t00);
  g = fmaf(w10, numer_g(t10), g);
  g = fmaf(w01, numer_g(t01), g);
  g = fmaf(w11, numer_g(t11), g);
  float b = w00 * numer_b(t00);
  b = fmaf(w10, numer_b(t10), b);
  b = fmaf(w01, numer_b(t01), b);
  b = fmaf(w11, numer_b(t11), b);
  return make_float3(r * kInvDenRB, g * kInvDenG, b * kInvDenRB);
}

// One level sampled with direct block fetches (no staging).
__device__ __forceinline__ float3 sample_bc1_direct(const LevelArgs &L, float u, float v, int mode) {
  const Taps t = tap_coords(u, v, L, mode);
  return blend_numer(bc1_texel_global(L, t.i0, t.j0), bc1_texel_global(L, t.i1, t.j0),
                     bc1_texel_global(L, t.i0, t.j1), bc1_texel_global(L, t.i1, t.j1), t.fx, t.fy);
}

// One level of float latents.
__device__ __forceinline__ float3 sample_f32(const LevelArgs &L, float u, float v, int mode) {
  const Taps t = tap_coords(u, v, L, mode);
  const float gx = 1.0f - t.fx, gy = 1.0f - t.fy;
  const float w[4] = {gx * gy, t.fx * gy, gx * t.fy, t.fx * t.fy};
  const int ii[4] = {t.i0, t.i1, t.i0, t.i1};
  const int jj[4] = {t.j0, t.j0, t.j1, t.j1};
  float3 c = make_float3(0.f, 0.f, 0.f);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float *p = L.grid + ((int64_t)jj[k] * L.w + ii[k]) * 3;
    c.x = fmaf(w[k], p[0], c.x);
    c.y = fmaf(w[k], p[1], c.y);
    c.z = fmaf(w[k], p[2], c.z);
  }
  return c;
}

__device__ __forceinline__ float3 sample_level(const LatArgs &lat, int k, float u, float v) {
  return lat.format == 0 ? sample_bc1_direct(lat.lv[k], u, v, lat.address)
                         : sample_f32(lat.lv[k], u, v, lat.address);
}

}  // namespace ntc
