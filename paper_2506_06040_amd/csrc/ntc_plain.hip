// Plain FP32 decode (one pixel per lane, scalar FMAs: the analogue of the
// paper's "software FMA" path of Table 2), the FP8 range calibration that
// shares it, the BC1 texel export, small fill kernels and the weight
// packers.
#include <hip/hip_runtime.h>

#include "ntc_device.hpp"
#include "ntc_internal.hpp"

namespace ntc {

// ---------------------------------------------------------------------------
// Packed layouts
// ---------------------------------------------------------------------------
static inline uint32_t align_up(size_t v, size_t a) { return (uint32_t)((v + a - 1) / a * a); }

PackLayout pack_layout(const MlpShape &s, int compute) {
  PackLayout L{};
  size_t off = 0;
  const int Ln = s.n_layers;
  if (compute == 0) {  // FP32
    L.elem_bytes = 4;
    for (int l = 0; l < Ln; ++l) {
      const int rows = (l == Ln - 1) ? 16 : s.hid;
      const int cols = (l == 0) ? 16 : s.hid;
      L.rows_pad[l] = rows;
      L.cols_pad[l] = cols;
      L.w_off[l] = align_up(off, 256);
      off = L.w_off[l] + (size_t)rows * cols * 4;
      L.b_off[l] = align_up(off, 256);
      off = L.b_off[l] + (size_t)rows * 4;
    }
  } else {
    // 32x32 matrix-core tiles: M-tiles of 32 output rows; K-steps of 16
    // inputs (FP16, 8 per lane) or 64 inputs (E4M3, 32 per lane).
    const bool f8 = compute == 3;
    L.elem_bytes = f8 ? 1 : 2;
    L.frag_elems = f8 ? 32 : 8;
    const int kstep = f8 ? 64 : 16;
    const size_t frag = 64 * (size_t)L.frag_elems * (size_t)L.elem_bytes;
    for (int l = 0; l < Ln; ++l) {
      const int rows = (l == Ln - 1) ? s.n_out : s.hid;
      const int cols = (l == 0) ? s.in_dim : s.hid;
      L.mt[l] = (rows + 31) / 32;
      L.kc[l] = (cols + kstep - 1) / kstep;
      L.w_off[l] = align_up(off, 256);
      off = L.w_off[l] + (size_t)L.mt[l] * L.kc[l] * frag;
      L.b_off[l] = align_up(off, 256);
      off = L.b_off[l] + (size_t)L.mt[l] * 2 * 16 * sizeof(float);
    }
  }
  L.scale_off = align_up(off, 256);
  off = L.scale_off + 4 * kMaxLayers * sizeof(float);
  L.exp_off = align_up(off, 256);
  off = L.exp_off + kMaxLayers * 64 * sizeof(int32_t);
  L.total = align_up(off, 256);
  return L;
}

struct PackArgs {
  MlpPtrs p;
  MlpShape s;
  PackLayout lay;
  const float *act_amax;
  uint8_t *packed;
  int compute;
};

// Input index fed to K-slot (lane half h, element e) of the first layer:
// half 0 carries [L0 r, g, b, u, L1 r, g, b, v], half 1 [L2 r, g, b, -,
// L3 r, g, b, -] (a level's three channels and one more slot per group of
// four, so that a level's packed FP16 sample (r, g), (b, x) is two operand
// dwords as it stands).
__device__ __forceinline__ int feature_col(int n_levels, int h, int e) {
  if ((e & 3) < 3) {
    const int lvl = 2 * h + (e >> 2);
    return lvl < n_levels ? 3 * lvl + (e & 3) : -1;
  }
  if (h == 0) return 3 * n_levels + (e >> 2);  // u, v
  return -1;
}

// Source column of element e of lane half h in K-step c of layer l, or -1 for
// padding. Hidden layers take their K order from the accumulator layout of
// the previous layer (lane half h holds rows 8 j + 4 h + r, j, r < 4, of each
// 32-row tile):
//   FP16, K-step 16: element e is unit 32 (c/2) + 16 (c%2) + 8 (e/4) + 4 h + e%4
//   E4M3, K-step 64: element e is unit 32 (2c + e/16) + 8 ((e%16)/4) + 4 h + e%4
// With NTC_FOLD_BIAS the first layer's K-slots 3 and 7 of lane half 1 (fed
// with 1 by the decode) take the bias: kColBiasHi, kColBiasLo.
constexpr int kColBiasHi = -2, kColBiasLo = -3;

__device__ __forceinline__ int frag_source_col(const MlpShape &s, bool f8, int l, int c, int h, int e) {
  if (l == 0) {
    if (f8) return e >= 8 ? -1 : feature_col((s.in_dim - 2) / 3, h, e);
    if (NTC_FOLD_BIAS && h == 1 && (e & 3) == 3) return e == 3 ? kColBiasHi : kColBiasLo;
    return feature_col((s.in_dim - 2) / 3, h, e);
  }
  int u;
  if (f8)
    u = 32 * (2 * c + (e >> 4)) + 8 * ((e & 15) >> 2) + 4 * h + (e & 3);
  else
    u = 32 * (c >> 1) + 16 * (c & 1) + 8 * (e >> 2) + 4 * h + (e & 3);
  return u < s.hid ? u : -1;
}

// Largest power of two <= x (x > 0 and finite).
__device__ __forceinline__ float pow2_floor(float x) {
  x = fminf(fmaxf(x, 0x1p-100f), 0x1p100f);  // keeps the E8M0 exponents in range
  return ldexpf(1.0f, __builtin_amdgcn_frexp_expf(x) - 1);
}

// Scales of the E4M3 image, powers of two: s_w = 2^floor(log2(448 /
// max|W_l|)); for the first layer's inputs s_a = 2^floor(log2(448 /
// max(act_amax[0], 1))) (BC1 latent values reach 1 whatever the calibration
// saw, so a latent times s_a never leaves E4M3's range); for hidden
// activations s_a = 2^floor(log2(256 / act_amax[l])), because the decode
// clamps their scaled values to [0, 256] (ReLU and clamp as one FP16
// conversion of the value / 256, then the scaled FP16 -> E4M3 conversion).
// Stored per layer as (s_a, epilogue, s_w). The epilogue factor maps the
// accumulator of layer l to the next layer's scaled input / 256 (s_a(l + 1)
// / (256 s_w s_a)) or, for the last layer, to the pre-activation (1 / (s_w
// s_a)); being a power of two, the decode applies it as the E8M0 block
// scale of the layer's matrix instructions, and the packed bias is b s_w s_a
// times it.
__device__ __forceinline__ float act_scale(float am, int l) {
  if (l == 0) return pow2_floor(448.0f / fmaxf(am, 1.0f));
  return am > 0.f ? pow2_floor(256.0f / am) : 1.0f;
}

__global__ void pack_scales_kernel(PackArgs a) {
  const int l = blockIdx.x;
  const int rows = a.p.dims[l + 1], cols = a.p.dims[l];
  float m = 0.f;
  for (int i = threadIdx.x; i < rows * cols; i += blockDim.x) m = fmaxf(m, fabsf(a.p.W[l][i]));
  __shared__ float red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float wm = red[0];
    const float sw = wm > 0.f ? pow2_floor(448.0f / wm) : 1.0f;
    const float sa = act_scale(a.act_amax[l], l);
    float epi;
    if (l + 1 < a.s.n_layers) {
      epi = act_scale(a.act_amax[l + 1], l + 1) / (256.0f * sw * sa);
    } else {
      epi = 1.0f / (sw * sa);
    }
    float *sc = (float *)(a.packed + a.lay.scale_off);
    sc[3 * l + 0] = sa;
    sc[3 * l + 1] = epi;
    sc[3 * l + 2] = sw;
  }
}

// FP16 image: per-neuron power-of-two scales that let the matrix-core decode
// apply ReLU and the FP16 conversion in one instruction (conversion with
// the [0, 1] clamp). Hidden neuron i of layer l is stored as its activation
// times 2^-e(l, i), with e chosen so that the scaled pre-activation cannot
// exceed 1 when every input lies in [0, 1] (BC1 latent values always do;
// the coordinate features do when u, v are in [0, 1]): an interval bound
// over that box, with inputs of hidden layers in [0, 2^e] of the previous
// layer, plus a margin for FP16 products and FP32 sums (2^-8 of the
// absolute sum, far above their rounding). The weights of layer l are then
// W(i, j) 2^(e(l-1, j) - e(l, i)) and its bias b(i) 2^-e(l, i) (e = 0 for
// the network inputs and outputs): powers of two, so the network computes
// the same function and only the placement of FP16 rounding in the
// subnormal range changes. When a bound exceeds 2^kMaxClampExp the image
// keeps e = 0 everywhere and the flag (first scale word) is 0, which sends
// every span to the max-based ReLU.
constexpr int kMaxClampExp = 10;

__device__ __forceinline__ int bound_exp(double u) {
  if (!(u > 1.0)) return u == u ? 0 : kMaxClampExp + 1;
  int k;
  const double m = frexp(u, &k);  // u = m 2^k, m in [0.5, 1)
  return m == 0.5 ? k - 1 : k;
}

__global__ __launch_bounds__(64) void pack_bounds_kernel(PackArgs a) {
  __shared__ int e_prev[64];
  __shared__ int bad;
  const int i = threadIdx.x;
  const int Ln = a.s.n_layers;
  int *ex = reinterpret_cast<int *>(a.packed + a.lay.exp_off);
  e_prev[i] = 0;
  if (i == 0) bad = 0;
  __syncthreads();
  for (int l = 0; l + 1 < Ln; ++l) {
    const int rows = a.p.dims[l + 1], cols = a.p.dims[l];
    int e = 0;
    if (i < rows) {
      const double b = a.p.b[l][i];
      double hi = b, mag = fabs(b);
      for (int j = 0; j < cols; ++j) {
        const double w = a.p.W[l][(int64_t)i * cols + j];
        const double x = ldexp(1.0, e_prev[j]);
        if (w > 0.0) hi += w * x;
        mag += fabs(w) * x;
      }
      e = bound_exp(hi + ldexp(mag, -8) + ldexp(1.0, -20));
      if (e > kMaxClampExp) bad = 1;
    }
    __syncthreads();
    e_prev[i] = e;
    ex[l * 64 + i] = e;
    __syncthreads();
  }
  // The output layer keeps e = 0, so its weights take the whole factor
  // 2^e(j) of their input neuron j: the image is only usable if every such
  // weight stays finite in FP16 (|W| 2^e(j) <= 2^15 < 65504, leaving room
  // for the conversion's rounding); otherwise it stays unscaled.
  {
    const int rows = a.p.dims[Ln], cols = a.p.dims[Ln - 1];
    if (i < cols) {
      double m = 0.0;
      for (int r = 0; r < rows; ++r) m = fmax(m, fabs((double)a.p.W[Ln - 1][(int64_t)r * cols + i]));
      if (!(ldexp(m, e_prev[i]) <= 32768.0)) bad = 1;
    }
    __syncthreads();
  }
  const bool ok = bad == 0;
  for (int l = Ln - 1; l < kMaxLayers; ++l) ex[l * 64 + i] = 0;
  if (!ok)
    for (int l = 0; l + 1 < Ln; ++l) ex[l * 64 + i] = 0;
  if (i == 0) reinterpret_cast<float *>(a.packed + a.lay.scale_off)[0] = ok ? 1.0f : 0.0f;
}

__device__ __forceinline__ uint8_t to_e4m3(float v) {
  v = fminf(fmaxf(v, -448.0f), 448.0f);
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xFF);
}

// One thread per element of the image (weights, then biases).
__global__ void pack_kernel(PackArgs a, int64_t n_w_elems, int64_t n_elems) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elems) return;
  const MlpShape &s = a.s;
  const PackLayout &L = a.lay;
  const int Ln = s.n_layers;
  const float *sc = (const float *)(a.packed + L.scale_off);
  if (a.compute == 0) {
    // FP32 image: walk layers
    int64_t r = e;
    for (int l = 0; l < Ln; ++l) {
      const int64_t nw = (int64_t)L.rows_pad[l] * L.cols_pad[l];
      const int64_t nb = L.rows_pad[l];
      const int rows = a.p.dims[l + 1], cols = a.p.dims[l];
      if (r < nw) {
        const int row = (int)(r / L.cols_pad[l]), col = (int)(r % L.cols_pad[l]);
        float v = 0.f;
        if (row < rows && col < cols) v = a.p.W[l][(int64_t)row * cols + col];
        ((float *)(a.packed + L.w_off[l]))[r] = v;
        return;
      }
      r -= nw;
      if (r < nb) {
        const int row = (int)r;
        ((float *)(a.packed + L.b_off[l]))[r] = row < rows ? a.p.b[l][row] : 0.f;
        return;
      }
      r -= nb;
    }
    return;
  }
  if (e < n_w_elems) {
    int64_t r = e;
    const bool f8 = a.compute == 3;
    const int E = L.frag_elems;
    for (int l = 0; l < Ln; ++l) {
      const int64_t nl = (int64_t)L.mt[l] * L.kc[l] * 64 * E;
      if (r < nl) {
        const int el = (int)(r % E);
        const int lane = (int)((r / E) & 63);
        const int64_t fr = r / (64 * E);  // frag index = m * kc + c
        const int c = (int)(fr % L.kc[l]), m = (int)(fr / L.kc[l]);
        const int row = 32 * m + (lane & 31);
        const int col = frag_source_col(s, f8, l, c, lane >> 5, el);
        const int rows = a.p.dims[l + 1], cols = a.p.dims[l];
        float v = 0.f;
        if (row < rows && col >= 0 && col < cols) v = a.p.W[l][(int64_t)row * cols + col];
        if (col <= kColBiasHi) {
          // first-layer bias as two weights of the constant-1 slots: the
          // operand-type value nearest the bias, then the nearest value to
          // the remainder (exact in FP32)
          float bv = row < rows ? a.p.b[0][row] : 0.f;
          if (a.compute == 1) bv = ldexpf(bv, -((const int *)(a.packed + L.exp_off))[row < 64 ? row : 0]);
          if (a.compute == 2) {
            const __bf16 hi = (__bf16)bv;
            ((__bf16 *)(a.packed + L.w_off[l]))[r] = col == kColBiasHi ? hi : (__bf16)(bv - (float)hi);
          } else {
            const _Float16 hi = (_Float16)bv;
            ((_Float16 *)(a.packed + L.w_off[l]))[r] = col == kColBiasHi ? hi : (_Float16)(bv - (float)hi);
          }
          return;
        }
        if (f8) {
          (a.packed + L.w_off[l])[r] = to_e4m3(v * sc[3 * l + 2]);
        } else if (a.compute == 2) {
          ((__bf16 *)(a.packed + L.w_off[l]))[r] = (__bf16)v;
        } else {
          const int *ex = (const int *)(a.packed + L.exp_off);
          const int e_in = (l > 0 && col >= 0) ? ex[(l - 1) * 64 + col] : 0;
          const int e_out = (l + 1 < Ln && row < 64) ? ex[l * 64 + row] : 0;
          ((_Float16 *)(a.packed + L.w_off[l]))[r] = (_Float16)ldexpf(v, e_in - e_out);
        }
        return;
      }
      r -= nl;
    }
    return;
  }
  // bias fragments: [m][h][16] floats, element 4 j + r = row 32 m + 8 j + 4 h + r
  int64_t r = e - n_w_elems;
  for (int l = 0; l < Ln; ++l) {
    const int64_t nb = (int64_t)L.mt[l] * 32;
    if (r < nb) {
      const int m = (int)(r / 32), h = (int)((r / 16) & 1), q = (int)(r & 15);
      const int row = 32 * m + 8 * (q >> 2) + 4 * h + (q & 3);
      const int rows = a.p.dims[l + 1];
      float v = row < rows ? a.p.b[l][row] : 0.f;
      if (a.compute == 3) v = v * (sc[3 * l + 2] * sc[3 * l + 0] * sc[3 * l + 1]);
      if (a.compute == 1 && l + 1 < Ln) v = ldexpf(v, -((const int *)(a.packed + L.exp_off))[l * 64 + row]);
      ((float *)(a.packed + L.b_off[l]))[r] = v;
      return;
    }
    r -= nb;
  }
}

hipError_t launch_pack(const MlpShape &s, const MlpPtrs &p, int compute, const float *act_amax,
                       uint8_t *packed, const PackLayout &lay, hipStream_t st) {
  PackArgs a;
  a.p = p;
  a.s = s;
  a.lay = lay;
  a.act_amax = act_amax;
  a.packed = packed;
  a.compute = compute;
  int64_t n_w = 0, n_all = 0;
  if (compute == 0) {
    for (int l = 0; l < s.n_layers; ++l) n_all += (int64_t)lay.rows_pad[l] * lay.cols_pad[l] + lay.rows_pad[l];
    n_w = n_all;
  } else {
    for (int l = 0; l < s.n_layers; ++l) n_w += (int64_t)lay.mt[l] * lay.kc[l] * 64 * lay.frag_elems;
    n_all = n_w;
    for (int l = 0; l < s.n_layers; ++l) n_all += (int64_t)lay.mt[l] * 32;
  }
  if (compute == 3 || compute == 1) {
    if (compute == 3)
      hipLaunchKernelGGL(pack_scales_kernel, dim3(s.n_layers), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL(pack_bounds_kernel, dim3(1), dim3(64), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int bs = 256;
  const int64_t grid = (n_all + bs - 1) / bs;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)grid), dim3(bs), 0, st, a, n_w, n_all);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain FP32 decode
// ---------------------------------------------------------------------------
__device__ __forceinline__ void atomic_max_nonneg(float *addr, float v) {
  // non-negative IEEE floats order like their bit patterns
  atomicMax(reinterpret_cast<unsigned int *>(addr), __float_as_uint(v));
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

template <int HID, bool CALIB>
// The packed image comes as its own read-only, non-aliasing argument: its
// loads are then uniform and unclobbered, and the compiler reads the weights
// through the scalar cache (one load for the whole wavefront) instead of
// once per lane.
__global__ __launch_bounds__(256) void decode_plain_kernel(DecodeArgs a, const float *__restrict__ wp,
                                                           float *__restrict__ amax) {
  const int n_levels = a.lat.n_levels;
  const int n_layers = a.n_layers;
  const int n_out = a.n_out;
  float am[kMaxLayers];
#pragma unroll
  for (int l = 0; l < kMaxLayers; ++l) am[l] = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int iter = 0;  // wavefront-uniform iteration count: salt of opaque_zero
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += stride, iter += 4) {
    // weights read through a per-iteration opaque offset, so that their
    // scalar loads stay in the loop instead of being hoisted out of it into
    // scalar registers that spill into vector lanes
    const float *wpi = wp + opaque_zero(iter);
    const float2 uv = a.uv[p];
    float x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = 0.f;
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) {
      if (k < n_levels) {
        const float3 c = sample_level(a.lat, k, uv.x, uv.y);
        x[3 * k] = c.x;
        x[3 * k + 1] = c.y;
        x[3 * k + 2] = c.z;
      }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (k == 3 * n_levels) x[k] = uv.x;
      if (k == 3 * n_levels + 1) x[k] = uv.y;
    }
    if (CALIB) {
#pragma unroll
      for (int k = 0; k < 16; ++k) am[0] = fmaxf(am[0], fabsf(x[k]));
    }
    float h[HID];
    {
      const float *W = wpi + a.lay.w_off[0] / 4;
      const float *b = wpi + a.lay.b_off[0] / 4;
#pragma unroll
      for (int o = 0; o < HID; ++o) {
        float acc = b[o];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc = fmaf(W[o * 16 + k], x[k], acc);
        h[o] = fmaxf(acc, 0.f);
      }
    }
    for (int l = 1; l < n_layers - 1; ++l) {
      if (CALIB) {
#pragma unroll
        for (int k = 0; k < HID; ++k) am[l] = fmaxf(am[l], h[k]);
      }
      const float *W = wpi + a.lay.w_off[l] / 4;
      const float *b = wpi + a.lay.b_off[l] / 4;
      float h2[HID];
#pragma unroll
      for (int o = 0; o < HID; ++o) {
        float acc = b[o];
#pragma unroll
        for (int k = 0; k < HID; ++k) acc = fmaf(W[o * HID + k], h[k], acc);
        h2[o] = fmaxf(acc, 0.f);
      }
#pragma unroll
      for (int o = 0; o < HID; ++o) h[o] = h2[o];
    }
    if (CALIB) {
#pragma unroll
      for (int k = 0; k < HID; ++k) am[n_layers - 1] = fmaxf(am[n_layers - 1], h[k]);
      continue;  // calibration only needs the layer inputs
    }
    const float *W = wpi + opaque_zero(iter + 1) + a.lay.w_off[n_layers - 1] / 4;
    const float *b = wpi + opaque_zero(iter + 2) + a.lay.b_off[n_layers - 1] / 4;
#pragma unroll
    for (int o = 0; o < 16; ++o) {
      if (o < n_out) {
        float acc = b[o];
#pragma unroll
        for (int k = 0; k < HID; ++k) acc = fmaf(W[o * HID + k], h[k], acc);
        const float f = 1.0f / (1.0f + expf(-acc));
        if (a.out_f16)
          reinterpret_cast<_Float16 *>(a.out)[p * n_out + o] = (_Float16)f;
        else
          reinterpret_cast<float *>(a.out)[p * n_out + o] = f;
      }
    }
  }
  if (CALIB) {
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) {
      if (l < n_layers) {
        const float m = wave_max(am[l]);
        if ((threadIdx.x & 63) == 0) atomic_max_nonneg(amax + l, m);
      }
    }
  }
}

template <int HID>
static hipError_t launch_plain_hid(const DecodeArgs &a, float *calib, int n_cus, hipStream_t st) {
  const int bs = 256;
  int64_t blocks = (a.n + bs - 1) / bs;
  const int64_t cap = (int64_t)n_cus * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  if (calib)
    hipLaunchKernelGGL((decode_plain_kernel<HID, true>), dim3((unsigned)blocks), dim3(bs), 0, st, a,
                       reinterpret_cast<const float *>(a.packed), calib);
  else
    hipLaunchKernelGGL((decode_plain_kernel<HID, false>), dim3((unsigned)blocks), dim3(bs), 0, st, a,
                       reinterpret_cast<const float *>(a.packed), calib);
  return hipGetLastError();
}

hipError_t launch_decode_plain(const DecodeArgs &a, const MlpShape &s, float *calib_amax, int n_cus,
                               hipStream_t st) {
  switch (s.hid) {
    case 16: return launch_plain_hid<16>(a, calib_amax, n_cus, st);
    case 32: return launch_plain_hid<32>(a, calib_amax, n_cus, st);
    case 64: return launch_plain_hid<64>(a, calib_amax, n_cus, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// BC1 texel export and fills
// ---------------------------------------------------------------------------
__global__ void bc1_texels_kernel(LevelArgs L, float *out, uint16_t *numer) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)L.w * L.h;
  if (t >= n) return;
  const int i = (int)(t % L.w), j = (int)(t / L.w);
  const uint32_t p = bc1_texel_global(L, i, j);
  const uint32_t nr = p & 255u, nb = (p >> 8) & 255u, ng = p >> 16;
  if (numer) {
    numer[t * 3 + 0] = (uint16_t)nr;
    numer[t * 3 + 1] = (uint16_t)ng;
    numer[t * 3 + 2] = (uint16_t)nb;
  }
  if (out) {
    // one rounding of the exact quotient (the double quotient of these small
    // integers is never a float32 rounding tie, so no double rounding)
    out[t * 3 + 0] = (float)((double)nr / 186.0);
    out[t * 3 + 1] = (float)((double)ng / 378.0);
    out[t * 3 + 2] = (float)((double)nb / 186.0);
  }
}

hipError_t launch_bc1_texels(const LevelArgs &L, float *out, uint16_t *numer, hipStream_t st) {
  const int64_t n = (int64_t)L.w * L.h;
  const int bs = 256;
  hipLaunchKernelGGL(bc1_texels_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, L, out, numer);
  return hipGetLastError();
}

__global__ void fill_f32_kernel(float *p, int64_t n, float v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  int64_t blocks = (n + bs - 1) / bs;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)blocks), dim3(bs), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace ntc
