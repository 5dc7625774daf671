// Matrix-core tile decode shared by the single-material and the batched
// kernels.
//
// A wavefront decodes spans of 64 ST pixels (ST = NTC_SPAN_TILES):
//   1. uv of the span (buffer loads, prefetched one span ahead); lane l owns
//      pixels 64 q + l.
//   2. Footprint: every tap index is a monotonic function of the coordinate,
//      so the span's extreme coordinates (wave reductions) give each level's
//      tap range; 16 lanes evaluate them at once (level x axis x min/max).
//   3. Staging (clamp addressing, footprint within the LDS region): whole
//      blocks covering the footprint, one item per texel row of a block
//      (4 texels), all levels numbered in one sequence so that a single
//      round of 64 lanes usually covers the span. Each item is decoded with
//      exact integer arithmetic and written as FP32 texels to LDS. Otherwise,
//      and for wrap addressing, taps fetch their blocks directly.
//   4. Sub-spans of 64 pixels: each lane samples all levels of its own pixel
//      (clamp-to-edge applied to the sampling position: tap clamped to
//      [0, n - 2], fraction to [0, 1]), converts its 16 feature slots to the
//      operand type and trades operand halves with the other lane half
//      (v_permlane32_swap), which gives the B operands of two 32-pixel
//      N-tiles.
//   5. MLP on 32x32 matrix-core tiles: weights are the A operand (32 output
//      rows per M-tile), FP32 accumulation initialised with the bias. The
//      32x32 accumulator leaves lane 32 h + n with rows 8 j + 4 h + r
//      (j, r < 4) of pixel n; the next layer's weight columns are permuted at
//      pack time so that those rows are exactly the K elements the lane must
//      supply as B operand. Layers chain in registers: only ReLU and the
//      conversion run in between.
//   6. Sigmoid (hardware exp2 / reciprocal) on the rows that hold outputs,
//      buffer stores whose range check drops pixels past the end.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "ntc_device.hpp"
#include "ntc_internal.hpp"

// Compile-time tuning of the matrix-core decode.
#ifndef NTC_WAVES_PER_SIMD  // occupancy the register allocation is held to
#define NTC_WAVES_PER_SIMD 2
#endif
#ifndef NTC_SPAN_TILES  // 64-pixel tiles staged together (64-wide nets, 4+ layers)
#define NTC_SPAN_TILES 4
#endif
#ifndef NTC_SPAN_TILES_SMALL  // the same for the other shapes
#define NTC_SPAN_TILES_SMALL 8
#endif
#ifndef NTC_WIDE_NT  // N-tiles per MLP pass of 64-wide nets with hidden layers
#define NTC_WIDE_NT 2
#endif
#ifndef NTC_STAGED_UNROLL  // unroll the staged sub-span loop (exact memory-wait counts)
#define NTC_STAGED_UNROLL 1
#endif
#define NTC_PRAGMA(x) _Pragma(#x)
#if NTC_STAGED_UNROLL
#define NTC_UNROLL_STAGED NTC_PRAGMA(unroll)
#else
#define NTC_UNROLL_STAGED NTC_PRAGMA(unroll 1)
#endif
#ifndef NTC_MLP_PRIO  // wave priority (0..3) while a wave runs its MLP
#define NTC_MLP_PRIO 2
#endif
#ifndef NTC_STORE_AUX  // cache policy of the output stores (2: non-temporal)
#define NTC_STORE_AUX 2
#endif

namespace ntc {
// 64-pixel tiles per span for an MLP shape. A longer span spreads the
// footprint reductions, staging records and partly filled staging passes
// over more pixels, which pays where the MLP leaves registers for the
// longer span's coordinates; 64-wide networks keep the shorter span with
// four or more layers (88+ VGPRs of weights and two N-tiles of
// accumulators) and with FP32 texels (the BF16 and E4M3 decodes).
constexpr int span_tiles_for(int hid, int n_layers, bool f16_texels) {
  return (hid >= 64 && (n_layers >= 4 || !f16_texels)) ? NTC_SPAN_TILES : NTC_SPAN_TILES_SMALL;
}
}  // namespace ntc
#ifndef NTC_UV_PREFETCH  // load the next span's uv during the current span
#define NTC_UV_PREFETCH 1
#endif


namespace ntc {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
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

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ half2_t relu_pk(float a, float b) {
  const f32x2 v = {a, b};
  const half2_t h = __builtin_convertvector(v, half2_t);
  const half2_t z = {(_Float16)0.0f, (_Float16)0.0f};
  return __builtin_elementwise_max(h, z);
}

// ReLU for activations known to be at most 1: the [0, 1] clamp, which the
// compiler folds into the conversion (v_cvt_pk_f16_f32 with the clamp bit).
__device__ __forceinline__ half2_t relu_unit_pk(float a, float b) {
  const f32x2 v = {a, b};
  const half2_t h = __builtin_convertvector(v, half2_t);
  const half2_t z = {(_Float16)0.0f, (_Float16)0.0f}, o = {(_Float16)1.0f, (_Float16)1.0f};
  return __builtin_elementwise_min(__builtin_elementwise_max(h, z), o);
}

// FP16 operands, 32x32x16 tiles: a K-step is 16 inputs, 8 halves per lane.
struct PrecF16 {
  using Frag = half8_t;
  static constexpr int KSTEP = 16;
  static constexpr bool kScaled = false;
  static constexpr bool kUnitReLU = true;  // packed image scaled for ReLU by clamp
  static constexpr bool kF16Tex = true;    // texels staged and blended as packed FP16
  static constexpr int kFeatDwords = 4;  // dwords of a fragment that carry features
  __device__ __forceinline__ static f32x16 mma(Frag a, Frag b, f32x16 c, int, const int (&)[2]) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static Frag features(const float (&x)[8], float) {
    Frag f;
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
      const f32x2 p = {x[i], x[i + 1]};
      const half2_t h = __builtin_convertvector(p, half2_t);
      f[i] = h[0];
      f[i + 1] = h[1];
    }
    return f;
  }
  // K-step c of the next layer = ReLU of accumulator rows 8 (c % 2) .. + 7
  // of M-tile c / 2. UNIT: the activations are at most 1 (scaled image,
  // coordinates inside the unit square), so ReLU is the [0, 1] clamp.
  template <int MT, int KS, bool UNIT>
  __device__ __forceinline__ static void next_operands(const f32x16 (&acc)[MT], Frag (&hb)[KS], float) {
#pragma unroll
    for (int c = 0; c < KS; ++c) {
      const f32x16 &v = acc[(c >> 1) % MT];
      const int o = 8 * (c & 1);
#pragma unroll
      for (int i = 0; i < 8; i += 2) {
        const half2_t h = UNIT ? relu_unit_pk(v[o + i], v[o + i + 1]) : relu_pk(v[o + i], v[o + i + 1]);
        hb[c][i] = h[0];
        hb[c][i + 1] = h[1];
      }
    }
  }
};

// BF16 operands, 32x32x16 tiles (same layout as FP16). ReLU acts on the
// converted pair: a BF16 value is negative exactly when its sign bit is set,
// so the signed 16-bit maximum with 0 (one packed instruction per pair)
// zeroes the negative halves; rounding to nearest keeps the sign, so this
// equals rounding the ReLU of the FP32 value.
__device__ __forceinline__ bf16x2_t relu_bf16_pk(float a, float b) {
  typedef short s16x2_t __attribute__((ext_vector_type(2)));
  const f32x2 v = {a, b};
  const s16x2_t h = __builtin_bit_cast(s16x2_t, __builtin_convertvector(v, bf16x2_t));
  const s16x2_t z = {0, 0};
  return __builtin_bit_cast(bf16x2_t, __builtin_elementwise_max(h, z));
}

struct PrecBF16 {
  using Frag = bf16x8_t;
  static constexpr int KSTEP = 16;
  static constexpr bool kScaled = false;
  static constexpr bool kUnitReLU = false;
  static constexpr bool kF16Tex = false;
  static constexpr int kFeatDwords = 4;
  __device__ __forceinline__ static f32x16 mma(Frag a, Frag b, f32x16 c, int, const int (&)[2]) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static Frag features(const float (&x)[8], float) {
    Frag f;
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
      const f32x2 p = {x[i], x[i + 1]};
      const bf16x2_t h = __builtin_convertvector(p, bf16x2_t);
      f[i] = h[0];
      f[i + 1] = h[1];
    }
    return f;
  }
  template <int MT, int KS, bool>
  __device__ __forceinline__ static void next_operands(const f32x16 (&acc)[MT], Frag (&hb)[KS], float) {
#pragma unroll
    for (int c = 0; c < KS; ++c) {
      const f32x16 &v = acc[(c >> 1) % MT];
      const int o = 8 * (c & 1);
#pragma unroll
      for (int i = 0; i < 8; i += 2) {
        const bf16x2_t h = relu_bf16_pk(v[o + i], v[o + i + 1]);
        hb[c][i] = h[0];
        hb[c][i + 1] = h[1];
      }
    }
  }
};

// Four values to E4M3 bytes (first value in byte 0): the scaled conversion
// gives E4M3(x / inv), inv a power of two, so the scaling is exact. It does
// not saturate (a result beyond 448 becomes NaN): callers keep x / inv in
// [-448, 448].
typedef short short2_t __attribute__((ext_vector_type(2)));
// The conversions write one half of their destination and keep the other;
// the first of a pair writes the low half of a register whose high half the
// second overwrites, so its kept half is left unspecified (no zeroing move).
__device__ __forceinline__ short2_t any_short2() {
  short2_t z;  // unset on purpose
  return z;
}
__device__ __forceinline__ int pack4_e4m3(float a, float b, float c, float d, float inv) {
  const short2_t lo = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(any_short2(), a, b, inv, false);
  const short2_t w = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(lo, c, d, inv, true);
  return __builtin_bit_cast(int, w);
}

// Hidden activations to E4M3: the accumulators hold the next layer's scaled
// input / 256, so ReLU and the upper clamp are the [0, 1] clamp of the FP16
// conversion (one instruction per pair), and the scaled FP16 -> E4M3
// conversion multiplies by 256 (values in [0, 256], never beyond E4M3's
// range): one instruction per activation in all.
__device__ __forceinline__ int pack4_relu_e4m3(float a, float b, float c, float d) {
  const float inv256 = 0x1p-8f;
  const short2_t lo = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(any_short2(), relu_unit_pk(a, b), inv256, false);
  const short2_t w = __builtin_amdgcn_cvt_scalef32_pk_fp8_f16(lo, relu_unit_pk(c, d), inv256, true);
  return __builtin_bit_cast(int, w);
}

// E4M3 operands, 32x32x64 tiles (full-rate scaled form with unit block
// scales): a K-step is 64 inputs, 32 bytes per lane.
struct PrecF8 {
  using Frag = i32x8;
  static constexpr int KSTEP = 64;
  static constexpr bool kScaled = true;
  static constexpr bool kUnitReLU = false;
  static constexpr bool kF16Tex = false;
  static constexpr int kFeatDwords = 2;
  // Format 0 = E4M3 for both operands. The weights' E8M0 block scale
  // (127 + p for 2^p) carries layer l's epilogue factor: byte l % 4 of
  // sc[l / 4]; the activations' is 127 = 2^0, byte 1 of sc[1]. (The scale
  // operands are vector registers; the byte is chosen by op_sel.) l is a
  // constant after unrolling.
  __device__ __forceinline__ static f32x16 mma(Frag a, Frag b, f32x16 c, int l, const int (&sc)[2]) {
    switch (l) {
      case 0: return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sc[0], 1, sc[1]);
      case 1: return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 1, sc[0], 1, sc[1]);
      case 2: return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 2, sc[0], 1, sc[1]);
      case 3: return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 3, sc[0], 1, sc[1]);
      default: return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sc[1], 1, sc[1]);
    }
  }
  // inv: the reciprocal of the first layer's input scale (features times
  // the scale stay within E4M3's range: see pixel_operands)
  __device__ __forceinline__ static Frag features(const float (&x)[8], float inv) {
    Frag f = {0, 0, 0, 0, 0, 0, 0, 0};
    f[0] = pack4_e4m3(x[0], x[1], x[2], x[3], inv);
    f[1] = pack4_e4m3(x[4], x[5], x[6], x[7], inv);
    return f;
  }
  // K-step c of the next layer: bytes 0..15 from all rows of M-tile 2c,
  // bytes 16..31 from M-tile 2c + 1 (zero when it does not exist). The
  // accumulators are already in the next layer's input scale / 256 (the
  // layer's matrix instructions applied it), so this is ReLU, clamp and the
  // conversion (pack4_relu_e4m3).
  template <int MT, int KS, bool>
  __device__ __forceinline__ static void next_operands(const f32x16 (&acc)[MT], Frag (&hb)[KS], float) {
#pragma unroll
    for (int c = 0; c < KS; ++c) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (2 * c + q < MT) {
          const f32x16 &v = acc[2 * c + q];
#pragma unroll
          for (int w = 0; w < 4; ++w)
            hb[c][4 * q + w] = pack4_relu_e4m3(v[4 * w], v[4 * w + 1], v[4 * w + 2], v[4 * w + 3]);
        } else {
#pragma unroll
          for (int w = 0; w < 4; ++w) hb[c][4 * q + w] = 0;
        }
      }
    }
  }
};

// Dword d of an operand fragment, and its replacement.
template <class P>
__device__ __forceinline__ unsigned dword_of(const typename P::Frag &f, int d) {
  if constexpr (std::is_same_v<typename P::Frag, bf16x8_t>) {
    return __builtin_bit_cast(u32x4_t, f)[d];
  } else if constexpr (P::kFeatDwords == 4) {
    const half2_t h2 = {f[2 * d], f[2 * d + 1]};
    return __builtin_bit_cast(unsigned, h2);
  } else {
    const int w = f[d];
    return (unsigned)w;
  }
}
template <class P>
__device__ __forceinline__ void set_dword(typename P::Frag &f, int d, unsigned w) {
  if constexpr (std::is_same_v<typename P::Frag, bf16x8_t>) {
    u32x4_t v = __builtin_bit_cast(u32x4_t, f);
    v[d] = w;
    f = __builtin_bit_cast(bf16x8_t, v);
  } else if constexpr (P::kFeatDwords == 4) {
    const half2_t h2 = __builtin_bit_cast(half2_t, w);
    f[2 * d] = h2[0];
    f[2 * d + 1] = h2[1];
  } else {
    f[d] = (int)w;
  }
}

// Minimum / maximum over the 16 lanes of a DPP row (row rotations). A
// rotation reads a valid lane everywhere, so bound_ctrl changes no value; it
// lets the compiler fold the move into the min / max (v_min_i32_dpp).
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
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

// Sigmoid on the hardware exp2 / reciprocal; sigmoid_nb(z, nb) is
// sigmoid(z + b) for nb = -log2(e) b.
constexpr float kLog2E = 1.4426950408889634f;
__device__ __forceinline__ float sigmoid_fast(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-kLog2E * z));
}
__device__ __forceinline__ float sigmoid_nb(float z, float nb) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(fmaf(z, -kLog2E, nb)));
}

// Register-resident weights of one MLP (32-row M-tiles, K-steps of the
// precision's width).
template <class P, int HID, int NL>
struct MfmaWeights {
  static constexpr int MT = (HID + 31) / 32;                  // M-tiles of a hidden layer
  static constexpr int KS = (HID + P::KSTEP - 1) / P::KSTEP;  // K-steps of a hidden input
  static constexpr int NH = NL > 2 ? NL - 2 : 1;
  using Frag = typename P::Frag;
  Frag w0[MT];
  Frag wh[NH][MT][KS];
  Frag wo[KS];
  float epi[kMaxLayers];  // E4M3: epilogue factor of each layer (a power of two), as loaded
  int escale[2];          // the same as E8M0 bytes (see PrecF8::mma; set by ready())
  float in_scale;   // E4M3: reciprocal of the first layer's input scale
  float unit_flag;  // FP16 image scaled for ReLU by clamp (1.0) or not (0.0), as loaded
  int unit_relu;    // the same, wave-uniform (set by ready())
  // output bias of accumulator rows 4 h + i (i < 4) of this lane's half h,
  // times -log2(e): the sigmoid's exponent is then one multiply-add
  // (NTC_FOLD_BIAS; rows 8 + 4 h + i of widths above 8 are read where used)
  float ob[4];

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
        for (int c = 0; c < KS; ++c) wh[h][m][c] = gload(fh + (m * KS + c) * 64 + lane);
    }
    const Frag *fo = reinterpret_cast<const Frag *>(packed + lay.w_off[NL - 1]);
#pragma unroll
    for (int c = 0; c < KS; ++c) wo[c] = gload(fo + c * 64 + lane);
    in_scale = 1.0f;
    unit_flag = 0.0f;
    unit_relu = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) ob[i] = 0.0f;
    if (NTC_FOLD_BIAS) {
      const float *bo = reinterpret_cast<const float *>(packed + lay.b_off[NL - 1]) + 16 * (lane >> 5);
#pragma unroll
      for (int i = 0; i < 4; ++i) ob[i] = -kLog2E * gload(bo + i);
    }
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) epi[l] = 1.0f;
    if (P::kUnitReLU) unit_flag = gload(reinterpret_cast<const float *>(packed + lay.scale_off));
    if (P::kScaled) {
      const float *sc = reinterpret_cast<const float *>(packed + lay.scale_off);
      in_scale = 1.0f / gload(sc);  // a power of two: exact
#pragma unroll
      for (int l = 0; l < NL; ++l) epi[l] = gload(sc + 3 * l + 1);
    }
  }
  // Wait for the loads here (an empty asm that reads every register). A
  // persistent loop entered with these loads still pending would carry that
  // state into its body and wait for the whole vector-memory counter there
  // on every iteration.
  __device__ __forceinline__ void ready() {
#if defined(__HIP_DEVICE_COMPILE__)  // the constraints exist for the GPU target only
#pragma unroll
    for (int m = 0; m < MT; ++m) asm volatile("" ::"v"(w0[m]));
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < KS; ++c) asm volatile("" ::"v"(wh[h][m][c]));
#pragma unroll
    for (int c = 0; c < KS; ++c) asm volatile("" ::"v"(wo[c]));
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) asm volatile("" ::"v"(epi[l]));
    asm volatile("" ::"v"(in_scale));
    asm volatile("" ::"v"(unit_flag));
#pragma unroll
    for (int i = 0; i < 4; ++i) asm volatile("" ::"v"(ob[i]));
#endif
    unit_relu = __builtin_amdgcn_readfirstlane(unit_flag != 0.0f ? 1 : 0);
    // 2^p = 0.5 * 2^(p + 1): frexp's exponent is p + 1
    int e[kMaxLayers];
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) e[l] = P::kScaled ? 126 + __builtin_amdgcn_frexp_expf(epi[l]) : 127;
    escale[0] = e[0] | (e[1] << 8) | (e[2] << 16) | (e[3] << 24);
    escale[1] = e[4] | (127 << 8);
  }
};

// Left/top tap along one axis, clamp-to-edge: the position x = u f + c
// (c = shift - 1/2) is limited to [0, cap] (cap = n - 2) and floored, the
// fraction is x minus that tap, limited to [0, 1]; so an edge sample puts
// weight 1 on the edge texel, which equals clamping both taps. The tap is a
// monotonic function of u, which is what lets a span's footprint be bounded
// from its extreme coordinates.
__device__ __forceinline__ float tap_floor(float u, float f, float c, float capf) {
  return floorf(__builtin_amdgcn_fmed3f(fmaf(u, f, c), 0.0f, capf));
}
__device__ __forceinline__ void clamp_tap(float u, float f, float c, float capf, int &i0, float &fr) {
  const float x = fmaf(u, f, c);
  const float t = floorf(__builtin_amdgcn_fmed3f(x, 0.0f, capf));
  i0 = (int)t;
  fr = __builtin_amdgcn_fmed3f(x - t, 0.0f, 1.0f);
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

// A texel as packed FP16 values (r, g) and (b, 1): 8 bytes in LDS. The
// constant 1 passes through the blend unchanged (every interpolation of two
// equal values returns them exactly), which fills the first-layer K-slots
// that carry the bias.
struct Tex16 {
  half2_t rg, b1;
};
__device__ __forceinline__ Tex16 tex16_of(float3 c) {
  const f32x2 a = {c.x, c.y}, b = {c.z, 1.0f};
  Tex16 t;
  t.rg = __builtin_convertvector(a, half2_t);
  t.b1 = __builtin_convertvector(b, half2_t);
  return t;
}
__device__ __forceinline__ uint2 tex16_bits(Tex16 t) {
  return make_uint2(__builtin_bit_cast(unsigned, t.rg), __builtin_bit_cast(unsigned, t.b1));
}
__device__ __forceinline__ Tex16 tex16_from(uint2 w) {
  Tex16 t;
  t.rg = __builtin_bit_cast(half2_t, w.x);
  t.b1 = __builtin_bit_cast(half2_t, w.y);
  return t;
}

// Bilinear blend of four FP16 texels in packed FP16 arithmetic: the top and
// bottom pairs interpolated by fx, then those two by fy (each interpolation a
// subtraction and a fused multiply-add per pair of channels). fx and fy are
// rounded to FP16 first.
__device__ __forceinline__ Tex16 lerp_tex16(Tex16 t00, Tex16 t10, Tex16 t01, Tex16 t11, float fx, float fy) {
  const f32x2 f = {fx, fy};
  const half2_t fh = __builtin_convertvector(f, half2_t);
  const half2_t x = {fh[0], fh[0]}, y = {fh[1], fh[1]};
  Tex16 top, bot, c;
  top.rg = __builtin_elementwise_fma(x, t10.rg - t00.rg, t00.rg);
  top.b1 = __builtin_elementwise_fma(x, t10.b1 - t00.b1, t00.b1);
  bot.rg = __builtin_elementwise_fma(x, t11.rg - t01.rg, t01.rg);
  bot.b1 = __builtin_elementwise_fma(x, t11.b1 - t01.b1, t01.b1);
  c.rg = __builtin_elementwise_fma(y, bot.rg - top.rg, top.rg);
  c.b1 = __builtin_elementwise_fma(y, bot.b1 - top.b1, top.b1);
  return c;
}

__device__ __forceinline__ float3 texel_direct(const uint2 *bc1, int bw, int i, int j) {
  const uint2 blk = gload2u(bc1 + (int64_t)(j >> 2) * bw + (i >> 2));
  return texel_f32(bc1_numer(blk.x, blk.y, (uint32_t)(((j & 3) << 2) | (i & 3))));
}

// ---------------------------------------------------------------------------
// Buffer resources: SGPR base + 32-bit offsets; accesses at or beyond
// num_records bytes read 0 / are dropped by the hardware.
// ---------------------------------------------------------------------------
constexpr int kBufferFlags = 0x00020000;  // gfx9-family raw buffer word 3

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufferFlags);
}

// Bias fragments of all layers, copied once per wave into LDS: per layer
// and M-tile, 16 floats for each lane half (rows 8 j + 4 h + r), so that a
// lane's bias is the initial value of its 32x32 accumulator.
template <int HID, int NL>
struct BiasLds {
  static constexpr int MT = (HID + 31) / 32;
  static constexpr int kCount = ((NL - 1) * MT + 1) * 8;  // float4 entries
  __device__ __forceinline__ static int off(int l, int m) { return (l * MT + m) * 8; }  // l < NL - 1
  __device__ __forceinline__ static int off_out() { return (NL - 1) * MT * 8; }
  __device__ __forceinline__ static void fill(f32x4 *dst, const uint8_t *packed, const PackLayout &lay, int lane) {
    for (int e = lane; e < kCount; e += 64) {
      const int l = e < off_out() ? e / (MT * 8) : NL - 1;
      const int r = e < off_out() ? e % (MT * 8) : e - off_out();
      dst[e] = gload(reinterpret_cast<const f32x4 *>(packed + lay.b_off[l]) + r);
    }
  }
  __device__ __forceinline__ static f32x16 get(const f32x4 *src, int e0, int h) {
    const f32x4 *p = src + e0 + 4 * h;
    const f32x4 a = p[0], b = p[1], c = p[2], d = p[3];
    return (f32x16){a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3], c[0], c[1], c[2], c[3], d[0], d[1], d[2], d[3]};
  }
};

// MLP over NT N-tiles of 32 pixels (N-tiles t0 .. t0 + NT - 1 of the span) and
// store. VEC4: the output-width class (see store_outputs).
template <class P, int HID, int NL, int NT, bool UNIT>
__device__ __forceinline__ void mlp_compute(const MfmaWeights<P, HID, NL> &W, const f32x4 *bias,
                                            const typename P::Frag (&bx)[NT], f32x16 (&z)[NT], int salt) {
  using BL = BiasLds<HID, NL>;
  using WT = MfmaWeights<P, HID, NL>;
  constexpr int MT = WT::MT;
  constexpr int KS = WT::KS;
  constexpr int NH = NL - 2;
  using Frag = typename P::Frag;
  const int h = (threadIdx.x & 63) >> 5;
  bias += opaque_zero(salt);

  // the first layer's bias is in its weights (FP16 / BF16) and the output
  // layer's is added by the sigmoid (NTC_FOLD_BIAS): those accumulators
  // start at 0
  constexpr bool kFold0 = NTC_FOLD_BIAS && !P::kScaled;
  const f32x16 zero = {};
  f32x16 acc[NT][MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const f32x16 bm = kFold0 ? zero : BL::get(bias, BL::off(0, m), h);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t][m] = P::mma(W.w0[m], bx[t], bm, 0, W.escale);
  }
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    Frag hb[NT][KS];
#pragma unroll
    for (int t = 0; t < NT; ++t) P::template next_operands<MT, KS, UNIT>(acc[t], hb[t], W.epi[k]);
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const f32x16 bm = BL::get(bias, BL::off(1 + k, m), h);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        f32x16 s = P::mma(W.wh[k][m][0], hb[t][0], bm, 1 + k, W.escale);
#pragma unroll
        for (int c = 1; c < KS; ++c) s = P::mma(W.wh[k][m][c], hb[t][c], s, 1 + k, W.escale);
        acc[t][m] = s;
      }
    }
  }
  Frag hb[NT][KS];
#pragma unroll
  for (int t = 0; t < NT; ++t) P::template next_operands<MT, KS, UNIT>(acc[t], hb[t], W.epi[NL - 2]);
  const f32x16 bo = NTC_FOLD_BIAS ? zero : BL::get(bias, BL::off_out(), h);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    f32x16 s = P::mma(W.wo[0], hb[t][0], bo, NL - 1, W.escale);
#pragma unroll
    for (int c = 1; c < KS; ++c) s = P::mma(W.wo[c], hb[t][c], s, NL - 1, W.escale);
    z[t] = s;
  }
}

// Output-width classes (template argument VEC4 of the store path): widths
// that are not a multiple of 4 (rows leave one by one or through LDS),
// multiples of 4 up to 8 (one group of four rows per lane and no branch) and
// multiples of 4 above 8 (a second group).
constexpr int kOutAny = 0, kOut4 = 1, kOut4x2 = 2;
__host__ __device__ constexpr int out_class(int n_out) { return (n_out & 3) ? kOutAny : (n_out <= 8 ? kOut4 : kOut4x2); }

// Sigmoid of the output pre-activations of NT N-tiles (N-tiles t0 .. t0 +
// NT - 1 of the span) and store. VEC4: the output-width class.
template <class P, int NT, int VEC4, bool IDX = false>
__device__ __forceinline__ void store_outputs(const DecodeArgs &a, __amdgpu_buffer_rsrc_t ors,
                                              const f32x16 (&z)[NT], const float (&ob)[4], int t0, int salt,
                                              int64_t first = 0, int span = 0, float *obuf = nullptr) {
  const int lane = (threadIdx.x & 63);
  const int h = lane >> 5;
  // Widths that are not a multiple of 4 store up to eight values per lane
  // and group one by one; their offsets depend only on the lane and the
  // width, and hoisted out of the persistent loop they would be held (and
  // spilled) across it. An opaque zero keeps them next to the stores.
  const int n = (lane & 31) + (VEC4 ? 0 : opaque_zero(salt));
  const int n_out = a.n_out;
  const int esz = a.out_f16 ? 2 : 4;
  // Row groups j (rows 8 j + 4 h .. + 3) that hold outputs for some lane:
  // the first always (its store is unconditional), the second when there are
  // more than 8 outputs (at most 16). The sigmoid of the second group reads
  // its inputs through an empty asm inside the branch, so that the compiler
  // does not evaluate its transcendentals ahead of the branch.
  const bool two_groups = VEC4 == kOut4 ? false : n_out > 8;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    // FP32 rows whose width is not a multiple of 4, tile of 32 pixels
    // complete: the rows go through obuf (32 x n_out floats, the tile's
    // output bytes in order) and leave as contiguous 16-byte stores
    const bool stg = !VEC4 && !IDX && obuf != nullptr && !a.out_f16 && span >= 32 * (t0 + t + 1);
    int pix = 32 * (t0 + t) + n;
    if constexpr (IDX) {
      // the output row of an indexed sample is its pixel in the image (ors
      // covers the whole image); samples past the span are dropped
      const int64_t r = pix < span ? (int64_t)a.pix[first + pix] : -1;
      pix = (int)((r >= 0 && r < a.img_px) ? r : a.img_px);  // one past the image: dropped
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j == 0 || two_groups) {
        f32x4 zj = {z[t][4 * j], z[t][4 * j + 1], z[t][4 * j + 2], z[t][4 * j + 3]};
        f32x4 nb = {ob[0], ob[1], ob[2], ob[3]};
        if (j > 0) {
          asm volatile("" : "+v"(zj));
          if (NTC_FOLD_BIAS) {
            // rows 8 + 4 h .. + 3: elements 4 .. 7 of half h of the packed
            // output bias fragment ([half][16] floats)
            nb = gload(reinterpret_cast<const f32x4 *>(a.packed + a.lay.b_off[a.n_layers - 1]) + 4 * h + 1);
            nb = nb * -kLog2E;
          }
        }
        // (widths that are not a multiple of 4: rows that are outputs for no
        // lane of the group are skipped; the test is wavefront-uniform)
        f32x4 f = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (VEC4 || 8 * j + i < n_out) f[i] = NTC_FOLD_BIAS ? sigmoid_nb(zj[i], nb[i]) : sigmoid_fast(zj[i]);
        const int row = 8 * j + 4 * h;
        // rows past the output width and pixels past the end go beyond the
        // buffer and are dropped by its range check
        const int off0 = (pix * n_out + row) * esz;
        if (stg) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (row + i < n_out) obuf[(lane & 31) * n_out + row + i] = f[i];
        } else if (VEC4 == kOut4 && !IDX) {
          // No branch on the output type: both stores are issued, the one
          // of the type not requested through a resource of zero size
          // (dropped by its range check), so that a staged span stays one
          // basic block.
          const int off32 = row < n_out ? (pix * n_out + row) * 4 : 0x7fffffff;
          const __amdgpu_buffer_rsrc_t r32 = a.out_f16 ? make_rsrc(nullptr, 0) : ors;
          const __amdgpu_buffer_rsrc_t r16 = a.out_f16 ? ors : make_rsrc(nullptr, 0);
          const half4_t hv = __builtin_convertvector(f, half4_t);
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, f),
                                                 r32, off32, 0, NTC_STORE_AUX);
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, hv),
                                                r16, (int)((unsigned)off32 >> 1), 0, NTC_STORE_AUX);
        } else if (VEC4) {
          const int off = row < n_out ? off0 : 0x7fffffff;
          if (a.out_f16) {
            const half4_t hv = __builtin_convertvector(f, half4_t);
            __builtin_amdgcn_raw_buffer_store_b64(
                __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, hv), ors, off, 0, NTC_STORE_AUX);
          } else {
            __builtin_amdgcn_raw_buffer_store_b128(
                __builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, f), ors, off, 0, NTC_STORE_AUX);
          }
        } else if (!a.out_f16) {
          // FP32 rows of any width: a lane's four values in one 16-byte
          // store (dword-aligned) where all four are outputs, the others one
          // by one. Whether some lane needs a store depends only on j and the
          // width, so stores that no lane needs are not issued.
          const bool full = row + 4 <= n_out;
          if (8 * j + 4 <= n_out)
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, f),
                                                   ors, full ? off0 : 0x7fffffff, 0, NTC_STORE_AUX);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const bool need0 = 8 * j + 4 > n_out && 8 * j + i < n_out;
            const bool need1 = 8 * j + 8 > n_out && 8 * j + 4 + i < n_out;
            if (need0 || need1) {
              // element copied to a scalar first: bit-casting a vector
              // element in place reads element 0 with this compiler
              const float fi = f[i];
              const int oi = (!full && row + i < n_out) ? off0 + i * 4 : 0x7fffffff;
              __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(fi), ors, oi, 0, NTC_STORE_AUX);
            }
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float fi = f[i];
            const int oi = (row + i < n_out) ? off0 + i * esz : 0x7fffffff;
            const _Float16 hi = (_Float16)fi;
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, hi), ors, oi, 0, NTC_STORE_AUX);
          }
        }
      }
    }
    if (stg) {
      // The wavefront's LDS accesses complete in order, so the reads see the
      // rows other lanes just wrote; the empty asm keeps the compiler from
      // moving LDS accesses across the exchange. 8 n_out chunks of 16 bytes
      // per tile.
      asm volatile("" ::: "memory");
      const int base = 128 * (t0 + t) * n_out;
      for (int c = lane; c < 8 * n_out; c += 64) {
        const float *src = obuf + 4 * c;
        const f32x4 v = {src[0], src[1], src[2], src[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), ors,
                                               base + 16 * c, 0, NTC_STORE_AUX);
      }
      asm volatile("" ::: "memory");
    }
  }
}

// MLP over NT N-tiles of 32 pixels (N-tiles t0 .. t0 + NT - 1 of the span) and
// store.
template <class P, int HID, int NL, int NT, int VEC4, bool UNIT, bool IDX = false>
__device__ __forceinline__ void mlp_store(const DecodeArgs &a, const MfmaWeights<P, HID, NL> &W,
                                          const f32x4 *bias, __amdgpu_buffer_rsrc_t ors,
                                          const typename P::Frag (&bx)[NT], int t0, int salt, int64_t first = 0,
                                          int span = 0, float *obuf = nullptr) {
  f32x16 z[NT];
  mlp_compute<P, HID, NL, NT, UNIT>(W, bias, bx, z, salt);
  store_outputs<P, NT, VEC4, IDX>(a, ors, z, W.ob, t0, salt, first, span, obuf);
}


// Parameters of the latent levels, one table per wave in LDS (the kernels
// read them from here on every span instead of keeping the kernel
// argument's fields of all levels live in scalar registers). Level k has
// three entries:
//   3 k     {w, shift_x - 1/2, w - 2, w}      axis x
//   3 k + 1 {h, shift_y - 1/2, h - 2, h}      axis y
//   3 k + 2 {blocks (low, high 32 bits), blocks per row, 0}
// (w - 2 and h - 2 as floats, the other integers as their bits). The footprint lanes and the per-pixel taps use
// the same values.
struct LevelTab {
  static constexpr int kLevelEntries = 3 * kMaxLevels;
  // followed by two staging records per level, rewritten on every span
  static constexpr int kCount = kLevelEntries + 2 * kMaxLevels;
  __device__ __forceinline__ static void fill(f32x4 *dst, const LatArgs &lat, int lane) {
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) {
      const LevelArgs &L = lat.lv[k];
      const unsigned long long p = (unsigned long long)L.bc1;
      const f32x4 ex = {L.fw, L.sx - 0.5f, (float)(L.w - 2), __int_as_float(L.w)};
      const f32x4 ey = {L.fh, L.sy - 0.5f, (float)(L.h - 2), __int_as_float(L.h)};
      const f32x4 eb = {__uint_as_float((unsigned)p), __uint_as_float((unsigned)(p >> 32)), __int_as_float(L.bw),
                        0.0f};
      if (lane == 0) {
        dst[3 * k] = ex;
        dst[3 * k + 1] = ey;
        dst[3 * k + 2] = eb;
      }
    }
  }
};

// A level's parameters as read from the table.
struct TabLevel {
  float fw, cx, fh, cy, wm2, hm2;
  int w, h, bw;
  const uint2 *bc1;
  __device__ __forceinline__ void read(const f32x4 *tab, int k) {
    const f32x4 ex = tab[3 * k], ey = tab[3 * k + 1], eb = tab[3 * k + 2];
    fw = ex[0];
    cx = ex[1];
    wm2 = ex[2];
    w = __float_as_int(ex[3]);
    fh = ey[0];
    cy = ey[1];
    hm2 = ey[2];
    h = __float_as_int(ey[3]);
    bc1 = (const uint2 *)(((unsigned long long)__float_as_uint(eb[1]) << 32) | __float_as_uint(eb[0]));
    bw = __float_as_int(eb[2]);
  }
};

// Taps (columns i0, i1, rows j0, j1) and fractions of one level with direct
// block fetches; `mode` 0 clamp, 1 wrap.
__device__ __forceinline__ void direct_taps(const TabLevel &L, float u, float v, int mode, int &i0, int &i1, int &j0,
                                            int &j1, float &fx, float &fy) {
  if (mode == 0) {
    clamp_tap(u, L.fw, L.cx, L.wm2, i0, fx);
    clamp_tap(v, L.fh, L.cy, L.hm2, j0, fy);
    i1 = i0 + 1;
    j1 = j0 + 1;
    return;
  }
  float x = fmaf(u, L.fw, L.cx);
  float y = fmaf(v, L.fh, L.cy);
  x = fminf(fmaxf(x, -16777216.0f), 16777216.0f);
  y = fminf(fmaxf(y, -16777216.0f), 16777216.0f);
  const float xf = floorf(x), yf = floorf(y);
  const int ix = (int)xf, iy = (int)yf;
  i0 = address_coord(ix, L.w, 1);
  i1 = address_coord(ix + 1, L.w, 1);
  j0 = address_coord(iy, L.h, 1);
  j1 = address_coord(iy + 1, L.h, 1);
  fx = x - xf;
  fy = y - yf;
}

// Sample of one level with direct block fetches (FP32 blend).
__device__ __forceinline__ float3 sample_direct_t(const TabLevel &L, float u, float v, int mode) {
  int i0, i1, j0, j1;
  float fx, fy;
  direct_taps(L, u, v, mode, i0, i1, j0, j1, fx, fy);
  return blend4(texel_direct(L.bc1, L.bw, i0, j0), texel_direct(L.bc1, L.bw, i1, j0),
                texel_direct(L.bc1, L.bw, i0, j1), texel_direct(L.bc1, L.bw, i1, j1), fx, fy);
}

// The same sample with FP16 texels and the packed FP16 blend (bit for bit
// what the staged path computes from its LDS copy of the texels).
__device__ __forceinline__ Tex16 sample_direct16(const TabLevel &L, float u, float v, int mode) {
  int i0, i1, j0, j1;
  float fx, fy;
  direct_taps(L, u, v, mode, i0, i1, j0, j1, fx, fy);
  return lerp_tex16(tex16_of(texel_direct(L.bc1, L.bw, i0, j0)), tex16_of(texel_direct(L.bc1, L.bw, i1, j0)),
                    tex16_of(texel_direct(L.bc1, L.bw, i0, j1)), tex16_of(texel_direct(L.bc1, L.bw, i1, j1)), fx, fy);
}

// uv of the ST pixels a lane owns in a span of 64 ST pixels (pixel 64 q +
// lane); lanes past the end repeat the span's last pixel, so every loaded
// coordinate belongs to the span.
template <int ST>
struct SpanUv {
  float u[ST], v[ST];
  __device__ __forceinline__ void load(const float2 *uv, int64_t first_px, int64_t end_px) {
    const int lane = (threadIdx.x & 63);
    const int64_t left = end_px - first_px;
    const int span = left < 64 * ST ? (int)left : 64 * ST;
    const __amdgpu_buffer_rsrc_t urs = make_rsrc(uv + first_px, (uint32_t)span * 8u);
#pragma unroll
    for (int q = 0; q < ST; ++q) {
      const int p = min(64 * q + lane, span - 1);
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(urs, p * 8, 0, 0);
      u[q] = __uint_as_float(w[0]);
      v[q] = __uint_as_float(w[1]);
    }
  }
  // Indexed samples: sample s is pixel pix[s] of a uv image of img_px pixels
  // (img_px * 8 < 2^32). An index outside the image reads (0, 0).
  __device__ __forceinline__ void load_idx(const float2 *uv_img, int64_t img_px, const int32_t *pix,
                                           int64_t first_px, int64_t end_px) {
    const int lane = (threadIdx.x & 63);
    const int64_t left = end_px - first_px;
    const int span = left < 64 * ST ? (int)left : 64 * ST;
    const __amdgpu_buffer_rsrc_t irs = make_rsrc(pix + first_px, (uint32_t)span * 4u);
    const __amdgpu_buffer_rsrc_t urs = make_rsrc(uv_img, (uint32_t)(img_px * 8));
#pragma unroll
    for (int q = 0; q < ST; ++q) {
      const int p = min(64 * q + lane, span - 1);
      const int idx = (int)__builtin_amdgcn_raw_buffer_load_b32(irs, p * 4, 0, 0);
      const uint32_t off = (idx >= 0 && (int64_t)idx < img_px) ? (uint32_t)idx * 8u : 0xFFFFFFF0u;
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(urs, off, 0, 0);
      u[q] = __uint_as_float(w[0]);
      v[q] = __uint_as_float(w[1]);
    }
  }
  template <bool IDX>
  __device__ __forceinline__ void load_any(const DecodeArgs &a, int64_t first_px, int64_t end_px) {
    if constexpr (IDX)
      load_idx(a.uv, a.img_px, a.pix, first_px, end_px);
    else
      load(a.uv, first_px, end_px);
  }
  // wait for the loads here (an empty asm that reads every coordinate)
  __device__ __forceinline__ void ready() const {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
    for (int q = 0; q < ST; ++q) asm volatile("" ::"v"(u[q]), "v"(v[q]));
#endif
  }
};

// Coordinates entering the clamp-mode taps: NaN becomes -2^20 and the range
// is limited to +-2^20, which changes no tap (any |u| >= 1 already sits on an
// edge for the level sizes the library accepts).
__device__ __forceinline__ float tap_coord(float u) { return fminf(fmaxf(u, -1048576.0f), 1048576.0f); }

// Signed integer with the order of a non-NaN float (negative floats have
// their magnitude bits flipped); the map is its own inverse. Reductions over
// these keys are integer DPP minimum / maximum (one instruction per step,
// with no NaN canonicalisation) finished on the scalar unit.
__device__ __forceinline__ int order_key(float f) {
  const int b = __float_as_int(f);
  return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float key_float(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }
__device__ __forceinline__ float wave_min_key(float v) {
  const int r = row_min_i(order_key(v));
  const int a = __builtin_amdgcn_readlane(r, 0), b = __builtin_amdgcn_readlane(r, 16);
  const int c = __builtin_amdgcn_readlane(r, 32), d = __builtin_amdgcn_readlane(r, 48);
  return key_float(min(min(a, b), min(c, d)));
}
__device__ __forceinline__ float wave_max_key(float v) {
  const int r = row_max_i(order_key(v));
  const int a = __builtin_amdgcn_readlane(r, 0), b = __builtin_amdgcn_readlane(r, 16);
  const int c = __builtin_amdgcn_readlane(r, 32), d = __builtin_amdgcn_readlane(r, 48);
  return key_float(max(max(a, b), max(c, d)));
}

// Operand exchange between the lane halves. Each lane computes all features
// of its own pixel: `lo` holds the K-slots of lane half 0, `hi` those of half
// 1. After the swap, `lo` is the B operand of the N-tile made of the pixels
// of lanes 0..31 and `hi` that of the pixels of lanes 32..63: the upper half
// of `lo` and the lower half of `hi` trade places (v_permlane32_swap).
template <class P>
__device__ __forceinline__ void swap_halves(typename P::Frag &lo, typename P::Frag &hi) {
#pragma unroll
  for (int d = 0; d < P::kFeatDwords; ++d) {
    const unsigned a = __builtin_bit_cast(unsigned, dword_of<P>(lo, d));
    const unsigned b = __builtin_bit_cast(unsigned, dword_of<P>(hi, d));
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    set_dword<P>(lo, d, r[0]);
    set_dword<P>(hi, d, r[1]);
  }
}

// Footprint and staging of one span whose lane coordinates are u, v (clamp
// addressing). The taps of every level are monotonic in (u, v), so the
// span's footprint on level k is spanned by the taps of the extreme
// coordinates, computed by 16 lanes in parallel (level, axis, min / max). If
// the footprints fit the LDS region (stage_cap texels), every texel in them
// is decoded once into `stage` (exact integer BC1 decode, scaled to FP32;
// F16TEX: then rounded to FP16, 8 bytes per texel, see Tex16) and
// the function returns true with kbw / kbase locating texel (i, j) of level
// k at j kbw[k] + i + kbase[k]. `srec` is this wave's staging record area
// (2 entries per level), `salt` a value that changes from span to span (see
// opaque_zero). in_unit (set when the span is staged): every u and v of the
// span lies in [0, 1] (NaN and infinities do not). interior: on every level
// the sampling position of every pixel of the span lies in [0, n - 2] on
// both axes, so the clamp of clamp_tap changes nothing.
template <int ST, bool F16TEX>
__device__ __forceinline__ bool stage_span(const DecodeArgs &a, const float (&u)[ST], const float (&v)[ST],
                                           f32x4 *stage, const f32x4 *ltab, f32x4 *srec, int salt,
                                           int (&kbw)[kMaxLevels], int (&kbase)[kMaxLevels], bool &in_unit,
                                           bool &interior) {
  const int lane = threadIdx.x & 63;
  in_unit = false;
  interior = false;
  if (a.lat.address != 0) return false;
  float umin = tap_coord(u[0]), umax = umin, vmin = tap_coord(v[0]), vmax = vmin;
#pragma unroll
  for (int q = 1; q < ST; ++q) {
    umin = fminf(umin, tap_coord(u[q]));
    umax = fmaxf(umax, tap_coord(u[q]));
    vmin = fminf(vmin, tap_coord(v[q]));
    vmax = fmaxf(vmax, tap_coord(v[q]));
  }
  // (tap_coord leaves no NaN)
  umin = wave_min_key(umin);
  umax = wave_max_key(umax);
  vmin = wave_min_key(vmin);
  vmax = wave_max_key(vmax);
  // the sanitised extremes: NaN became -2^20, infinities +-2^20
  in_unit = umin >= 0.0f && umax <= 1.0f && vmin >= 0.0f && vmax <= 1.0f;
  // lane 4 k + s (k < 4): tap index of an extreme coordinate on level k,
  // s = 0: left tap of umin, 1: left tap of umax, 2: top tap of vmin,
  // 3: top tap of vmax
  const int le = (lane >> 1) & 7;  // level le / 2, axis le % 2
  const f32x4 tb = (ltab + opaque_zero(salt))[3 * (le >> 1) + (le & 1)];
  const float ext = (lane & 2) ? ((lane & 1) ? vmax : vmin) : ((lane & 1) ? umax : umin);
  const int ti = (int)tap_floor(ext, tb[0], tb[1], tb[2]);
  // the positions are monotonic in the coordinate: the extremes decide
  const float raw = fmaf(ext, tb[0], tb[1]);
  interior = __builtin_amdgcn_ballot_w64(lane < 16 && !(raw >= 0.0f && raw <= tb[2])) == 0;
  // every lane of quad k receives the four values of level k
  const int qbx = __builtin_amdgcn_mov_dpp(ti, 0x00, 0xF, 0xF, false);
  const int qex = __builtin_amdgcn_mov_dpp(ti, 0x55, 0xF, 0xF, false);
  const int qby = __builtin_amdgcn_mov_dpp(ti, 0xAA, 0xF, 0xF, false);
  const int qey = __builtin_amdgcn_mov_dpp(ti, 0xFF, 0xF, 0xF, false);
  // Staged region of level k: the whole blocks spanning texel columns
  // [bx, ex + 1] (block columns col0 .. col0 + ncol - 1) on texel rows
  // [by, ey + 1]. A staging item is one texel row of one block (4 texels);
  // items are numbered level by level, row-major inside a level, and item
  // t owns staged texels 4 t .. 4 t + 3, so level k starts at texel
  // 4 ibase_k and its rows are 4 ncol_k texels wide.
  const int qcol0 = qbx >> 2;
  const int qncol = ((qex + 1) >> 2) - qcol0 + 1;
  const int qnrow = qey - qby + 2;
  // (levels past n_levels have a zero sampling scale: their footprint is
  // texels 0..1 x 0..1, two items)
  const int qitems = __mul24(qncol, qnrow);
  int kib[kMaxLevels], total = 0;
#pragma unroll
  for (int k = 0; k < kMaxLevels; ++k) {
    const int items = __builtin_amdgcn_readlane(qitems, 4 * k);
    const int col0 = __builtin_amdgcn_readlane(qcol0, 4 * k);
    const int by = __builtin_amdgcn_readlane(qby, 4 * k);
    kbw[k] = 4 * __builtin_amdgcn_readlane(qncol, 4 * k);
    kib[k] = total;
    kbase[k] = 4 * total - by * kbw[k] - 4 * col0;
    total += items;
  }
  if (4 * total > a.stage_cap) return false;
  // per-level staging records, written by the lead lane of each quad:
  // {first item, blocks per staged row, 1 / that, first block column}
  // and {first texel row, blocks per level row, block pointer}
  srec += opaque_zero(salt);
  if ((lane & 3) == 0 && lane < 4 * kMaxLevels) {
    const int k = lane >> 2;
    const int ib = k == 0 ? kib[0] : (k == 1 ? kib[1] : (k == 2 ? kib[2] : kib[3]));
    const f32x4 eb = (ltab + opaque_zero(salt))[3 * k + 2];
    srec[2 * k] = (f32x4){__int_as_float(ib), __int_as_float(qncol), __builtin_amdgcn_rcpf((float)qncol),
                          __int_as_float(qcol0)};
    srec[2 * k + 1] = (f32x4){__int_as_float(qby), eb[2], eb[0], eb[1]};
  }
  // item t: its block row (blocks, index word) and staged texels; the row
  // inside the level is (t - first + 1/2) / ncol rounded down, exact since
  // the reciprocal's relative error (~2^-22) moves a quotient that is at
  // least 1/(2 ncol) from an integer by < 1e-3 / ncol
  auto item_fetch = [&](int t, int &Y) {
    const int k = (t >= kib[1]) + (t >= kib[2]) + (t >= kib[3]);
    const f32x4 r0 = srec[2 * k], r1 = srec[2 * k + 1];
    const int tl = t - __float_as_int(r0[0]);
    const int ncol = __float_as_int(r0[1]);
    const int row = (int)(((float)tl + 0.5f) * r0[2]);
    const int col = tl - __mul24(row, ncol);
    Y = __float_as_int(r1[0]) + row;
    const uint2 *blk = (const uint2 *)(((unsigned long long)__float_as_uint(r1[3]) << 32) | __float_as_uint(r1[2]));
    // footprint rows and blocks lie inside the level
    return gload2u(blk + (__mul24(Y >> 2, __float_as_int(r1[1])) + __float_as_int(r0[3]) + col));
  };
  auto item_put = [&](int t, int Y, uint2 b) {
    const uint32_t pos = (uint32_t)(Y & 3) << 2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float3 val = texel_f32(bc1_numer(b.x, b.y, pos + i));
      if constexpr (F16TEX)
        reinterpret_cast<uint2 *>(stage)[4 * t + i] = tex16_bits(tex16_of(val));
      else
        stage[4 * t + i] = (f32x4){val.x, val.y, val.z, 0.0f};
    }
  };
  {
    int Y = 0;
    uint2 b = make_uint2(0u, 0u);
    if (lane < total) b = item_fetch(lane, Y);
    if (lane < total) item_put(lane, Y, b);
  }
  for (int t = lane + 64; t < total; t += 64) {
    int Y;
    const uint2 b = item_fetch(t, Y);
    item_put(t, Y, b);
  }
  return true;
}

// Operands of the pixel (uq, vq): its 16 feature slots (levels 0, 1 and
// (u, v) in the half-0 slots, levels 2, 3 in the half-1 slots), converted to
// the operand type and exchanged between the lane halves (swap_halves): bx[0]
// then feeds the N-tile of lanes 0..31's pixels, bx[1] that of lanes 32..63.
// Left/top tap and fraction of a staged pixel. INTERIOR (the span's
// positions lie in [0, n - 2]): floor and fraction of the position as they
// stand, which is what clamp_tap gives there; otherwise clamp_tap of the
// sanitised coordinate.
template <bool INTERIOR>
__device__ __forceinline__ void span_tap(float u, float f, float c, float capf, int &i0, float &fr) {
  if (INTERIOR) {
    const float x = fmaf(u, f, c);
    i0 = (int)x;  // x >= 0: truncation is the floor
    fr = __builtin_amdgcn_fractf(x);
  } else {
    clamp_tap(tap_coord(u), f, c, capf, i0, fr);
  }
}

// K-slots of the first layer (element e of lane half h): half 0 holds
// [L0 r, g, b, u, L1 r, g, b, v], half 1 [L2 r, g, b, c, L3 r, g, b, c],
// c = 1 in the slots of the first layer's bias (FP16 / BF16 with
// NTC_FOLD_BIAS) and 0 otherwise.
template <class P>
__device__ __forceinline__ void pixel_operands(float (&xl)[8], float (&xh)[8], float uq, float vq, float in_scale,
                                               typename P::Frag (&bx)[2]) {
  if constexpr (P::kScaled) {
    // E4M3: the coordinates saturate at the largest finite value (the
    // latents, at most 1, fit: their scale is at most 256)
    const float lim = 448.0f * in_scale;
    uq = __builtin_amdgcn_fmed3f(uq, -lim, lim);
    vq = __builtin_amdgcn_fmed3f(vq, -lim, lim);
  }
  xl[3] = uq;
  xl[7] = vq;
  xh[3] = (NTC_FOLD_BIAS && !P::kScaled) ? 1.0f : 0.0f;
  xh[7] = xh[3];
  bx[0] = P::features(xl, in_scale);
  bx[1] = P::features(xh, in_scale);
  swap_halves<P>(bx[0], bx[1]);
}

__device__ __forceinline__ void put_level(float (&xl)[8], float (&xh)[8], int k, float3 c) {
  float *x = k < 2 ? xl : xh;
  const int o = 4 * (k & 1);
  x[o] = c.x;
  x[o + 1] = c.y;
  x[o + 2] = c.z;
}

// FP16 operands from FP16 level samples (same K-slots as pixel_operands):
// each level's (r, g) and (b, 1) are fragment dwords as they stand; the pads
// of levels 0 and 1 take u and v.
__device__ __forceinline__ void operands16(const Tex16 (&c)[kMaxLevels], float uq, float vq, half8_t (&bx)[2]) {
  const f32x2 uvf = {uq, vq};
  const half2_t uv = __builtin_convertvector(uvf, half2_t);
  const half2_t bu = {c[0].b1[0], uv[0]}, bv = {c[1].b1[0], uv[1]};
  bx[0] = (half8_t){c[0].rg[0], c[0].rg[1], bu[0], bu[1], c[1].rg[0], c[1].rg[1], bv[0], bv[1]};
  bx[1] = (half8_t){c[2].rg[0], c[2].rg[1], c[2].b1[0], c[2].b1[1], c[3].rg[0], c[3].rg[1], c[3].b1[0], c[3].b1[1]};
  swap_halves<PrecF16>(bx[0], bx[1]);
}

// Operands of the pixel (uq, vq) from the staged texels.
template <class P, bool INTERIOR>
__device__ __forceinline__ void staged_operands(const DecodeArgs &a, const f32x4 *stage, const f32x4 *ltab,
                                                const int (&kbw)[kMaxLevels], const int (&kbase)[kMaxLevels],
                                                float uq, float vq, float in_scale, int salt,
                                                typename P::Frag (&bx)[2]) {
  if constexpr (P::kF16Tex) {
    const uint2 *s16 = reinterpret_cast<const uint2 *>(stage);
    Tex16 c[kMaxLevels];
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) {
      TabLevel Lk;
      Lk.read(ltab + opaque_zero(salt), k);
      int i0, j0;
      float fx, fy;
      span_tap<INTERIOR>(uq, Lk.fw, Lk.cx, Lk.wm2, i0, fx);
      span_tap<INTERIOR>(vq, Lk.fh, Lk.cy, Lk.hm2, j0, fy);
      int r = __mul24(j0, kbw[k]) + i0;
      asm("" : "+v"(r));
      const uint2 *t = s16 + kbase[k] + r;
      c[k] = lerp_tex16(tex16_from(t[0]), tex16_from(t[1]), tex16_from(t[kbw[k]]), tex16_from(t[kbw[k] + 1]), fx,
                        fy);
    }
    operands16(c, uq, vq, bx);
    return;
  }
  float xl[8], xh[8];
  // every level is sampled (levels past n_levels are harmless, see
  // to_lat_args): no branch, so a whole staged sub-span is one basic block
#pragma unroll
  for (int k = 0; k < kMaxLevels; ++k) {
    TabLevel Lk;
    Lk.read(ltab + opaque_zero(salt), k);
    int i0, j0;
    float fx, fy;
    span_tap<INTERIOR>(uq, Lk.fw, Lk.cx, Lk.wm2, i0, fx);
    span_tap<INTERIOR>(vq, Lk.fh, Lk.cy, Lk.hm2, j0, fy);
    // taps lie inside the staged region of the level; the row offset is
    // one multiply-add and the byte address one shift-add (the empty asm
    // keeps the compiler from distributing the shift over the sum)
    int r = __mul24(j0, kbw[k]) + i0;
    asm("" : "+v"(r));
    const f32x4 *t = stage + kbase[k] + r;
    const f32x4 t00 = t[0], t10 = t[1], t01 = t[kbw[k]], t11 = t[kbw[k] + 1];
    const float3 c = blend4(make_float3(t00[0], t00[1], t00[2]), make_float3(t10[0], t10[1], t10[2]),
                            make_float3(t01[0], t01[1], t01[2]), make_float3(t11[0], t11[1], t11[2]), fx, fy);
    put_level(xl, xh, k, c);
  }
  pixel_operands<P>(xl, xh, uq, vq, in_scale, bx);
}

// Operands of the pixel (uq, vq) with direct block fetches (footprint beyond
// the LDS region, or wrap addressing).
template <class P>
__device__ __forceinline__ void direct_operands(const DecodeArgs &a, const f32x4 *ltab, float uq, float vq,
                                                float in_scale, int salt, typename P::Frag (&bx)[2]) {
  if constexpr (P::kF16Tex) {
    Tex16 c[kMaxLevels];
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) {
      TabLevel Lk;
      Lk.read(ltab + opaque_zero(salt), k);
      c[k] = sample_direct16(Lk, uq, vq, a.lat.address);
    }
    operands16(c, uq, vq, bx);
    return;
  }
  float xl[8], xh[8];
#pragma unroll
  for (int k = 0; k < kMaxLevels; ++k) {
    TabLevel Lk;
    Lk.read(ltab + opaque_zero(salt), k);
    put_level(xl, xh, k, sample_direct_t(Lk, uq, vq, a.lat.address));
  }
  pixel_operands<P>(xl, xh, uq, vq, in_scale, bx);
}

// MLP and store of sub-span q of a span (two N-tiles of 32 pixels). UNIT:
// ReLU by the [0, 1] clamp (see PrecF16::next_operands).
template <class P, int HID, int NL, int VEC4, bool UNIT, bool IDX = false, bool PRIO = true>
__device__ __forceinline__ void subspan_mlp(const DecodeArgs &a, const MfmaWeights<P, HID, NL> &W, const f32x4 *bias,
                                            __amdgpu_buffer_rsrc_t ors, const typename P::Frag (&bx)[2], int q,
                                            int salt, int64_t first = 0, int span = 0, float *obuf = nullptr) {
  using Frag = typename P::Frag;
  // The other wave of the SIMD is usually sampling (vector work): issuing
  // this wave's matrix chain first lets the two overlap instead of both
  // waves reaching the MLP together. (PRIO false: the caller interleaves
  // its own sampling with the chain, and the priority changes would fence
  // the scheduler.)
  if (PRIO) __builtin_amdgcn_s_setprio(NTC_MLP_PRIO);
  // both N-tiles in one MLP pass when the weights leave room for two sets of
  // accumulators, otherwise one after the other
  if constexpr (HID >= 64 && NL >= 3 && NTC_WIDE_NT == 1) {
    const Frag b0[1] = {bx[0]}, b1[1] = {bx[1]};
    mlp_store<P, HID, NL, 1, VEC4, UNIT, IDX>(a, W, bias, ors, b0, 2 * q, salt, first, span, obuf);
    mlp_store<P, HID, NL, 1, VEC4, UNIT, IDX>(a, W, bias, ors, b1, 2 * q + 1, salt + 1, first, span, obuf);
  } else {
    mlp_store<P, HID, NL, 2, VEC4, UNIT, IDX>(a, W, bias, ors, bx, 2 * q, salt, first, span, obuf);
  }
  if (PRIO) __builtin_amdgcn_s_setprio(0);
}

// Output resource of a span: stores past `span` pixels are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_out(const DecodeArgs &a, int64_t first, int span) {
  const int esz = a.out_f16 ? 2 : 4;
  return make_rsrc(reinterpret_cast<const char *>(a.out) + first * a.n_out * esz, (uint32_t)(span * a.n_out * esz));
}

// Decode one span of up to 64 ST pixels starting at pixel `first` (uv
// already in uvs) and ending before end_px: footprint, staging, sampling,
// MLP, store. The uv of the next span (next_first < 0: none) is requested
// during this span, so that its latency overlaps the work of the span.
// obuf (2 KB of LDS, or nullptr): output staging of the FP32 rows of widths
// that are not a multiple of 4 (see store_outputs).
template <class P, int HID, int NL, int ST, int VEC4, bool IDX = false>
__device__ __forceinline__ void decode_span(const DecodeArgs &a, int64_t first, int64_t end_px, f32x4 *stage,
                                            const f32x4 *bias, f32x4 *ltab, const MfmaWeights<P, HID, NL> &W,
                                            SpanUv<ST> &uvs, int64_t next_first, int64_t next_end_px,
                                            float *obuf = nullptr) {
  using Frag = typename P::Frag;
  const int64_t left = end_px - first;
  const int span = left < 64 * ST ? (int)left : 64 * ST;
  const int span_salt = (int)first;
  // indexed samples write into the whole output image
  const __amdgpu_buffer_rsrc_t ors =
      IDX ? make_rsrc(a.out, (uint32_t)(a.img_px * a.n_out * (a.out_f16 ? 2 : 4))) : span_out(a, first, span);

  if (!NTC_UV_PREFETCH) uvs.template load_any<IDX>(a, first, end_px);
  float u[ST], v[ST];
#pragma unroll
  for (int q = 0; q < ST; ++q) {
    u[q] = uvs.u[q];
    v[q] = uvs.v[q];
  }
  int kbw[kMaxLevels], kbase[kMaxLevels];
  bool in_unit, interior;
  const bool staged = stage_span<ST, P::kF16Tex>(a, u, v, stage, ltab, ltab + LevelTab::kLevelEntries, span_salt,
                                                 kbw, kbase, in_unit, interior);

  // FP16: the staged path runs with ReLU by clamp, so it takes only spans
  // whose activations are known to be at most 1 (image scaled for it,
  // coordinates in the unit square); other spans take the direct path with
  // the max-based ReLU
  if (staged && (!P::kUnitReLU || (in_unit && W.unit_relu != 0))) {
    // The next span's uv is requested only now: the vector-memory counter
    // completes in order, so a load issued before the staging fetches would be
    // waited for together with them. After it come exactly the stores of the
    // ST sub-spans below (all of them run, also past the end of a short span,
    // whose stores the range check drops): that fixed count lets the wait
    // for these uv at the next span leave the stores in flight.
    if (NTC_UV_PREFETCH && next_first >= 0) uvs.template load_any<IDX>(a, next_first, next_end_px);
    // spans whose taps lie inside every level: no clamp on the tap
    // coordinates (same result, fewer instructions)
    if (interior) {
      NTC_UNROLL_STAGED
      for (int q = 0; q < ST; ++q) {
        Frag bx[2];
        staged_operands<P, true>(a, stage, ltab, kbw, kbase, u[q], v[q], W.in_scale, span_salt + q, bx);
        subspan_mlp<P, HID, NL, VEC4, P::kUnitReLU, IDX>(a, W, bias, ors, bx, q, span_salt + 2 * q, first, span,
                                                         obuf);
      }
    } else {
      NTC_UNROLL_STAGED
      for (int q = 0; q < ST; ++q) {
        Frag bx[2];
        staged_operands<P, false>(a, stage, ltab, kbw, kbase, u[q], v[q], W.in_scale, span_salt + q, bx);
        subspan_mlp<P, HID, NL, VEC4, P::kUnitReLU, IDX>(a, W, bias, ors, bx, q, span_salt + 2 * q, first, span,
                                                         obuf);
      }
    }
    return;
  }

  // direct block fetches; one sub-span at a time
#pragma unroll 1
  for (int q = 0; q < ST; ++q) {
    if (64 * q >= span) break;
    const float uq = u[0], vq = v[0];
#pragma unroll
    for (int i = 0; i + 1 < ST; ++i) {
      u[i] = u[i + 1];
      v[i] = v[i + 1];
    }
    Frag bx[2];
    direct_operands<P>(a, ltab, uq, vq, W.in_scale, q, bx);
    subspan_mlp<P, HID, NL, VEC4, false, IDX>(a, W, bias, ors, bx, q, 2 * q, first, span, obuf);
  }
  // the next span's uv, completed here: this path then leaves no pending
  // load behind and the wait state where the paths join is the staged one
  if (NTC_UV_PREFETCH && next_first >= 0) {
    uvs.template load_any<IDX>(a, next_first, next_end_px);
    uvs.ready();
  }
}

}  // namespace ntc
