// Backward of the FP32 decode for continuous latents (Sec. 3.2: gradients
// flow through the MLP into every latent element).
//
// Pass 1 (backward_mfma_kernel): per chunk of 32 samples, the forward is
// recomputed on the matrix cores (FP32 operands and accumulation), the
// deltas D_l = (W_{l+1}^T D_{l+1}) * [A_l > 0] (ReLU derivative 0 at 0) are
// products on the matrix cores too, and so are the weight gradients
// D_l A_l^T over the chunk's samples, accumulated in registers per
// wavefront. dx = W_0^T D_0, the gradient of the sample's latent features, is
// written to the workspace. Activations are never stored in global memory.
// At the end every wavefront writes its FP32 partial sums; a second kernel
// adds the partials of all wavefronts in FP64 and rounds once to FP32.
// Pass 2 (latent gradients, clamp addressing): the samples are grouped by
// spatial bin (a square of level-0 texels) with a counting sort; one
// workgroup per bin spreads dx onto the four bilinear taps of every level,
// adding into LDS copies of the texels the bin's samples can reach, and then
// adds those windows to the latent gradients with one atomic per texel and
// channel (taps outside a window fall back to a global atomic). With wrap
// addressing every tap is a global atomic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "ntc_device.hpp"
#include "ntc_internal.hpp"

namespace ntc {

// Number of MLP parameters, laid out per layer as W_l [rows][cols] then b_l.
static inline int n_params_of(const MlpShape &s) {
  int n = 0;
  int d[kMaxLayers + 1];
  d[0] = s.in_dim;
  for (int l = 1; l < s.n_layers; ++l) d[l] = s.hid;
  d[s.n_layers] = s.n_out;
  for (int l = 0; l < s.n_layers; ++l) n += d[l] * d[l + 1] + d[l + 1];
  return n;
}

// Matrix-core backward: workgroups of kBwdWaves wavefronts (one per SIMD),
// each wavefront taking kBwdChunk samples per step; one row of partial
// weight-gradient sums per wavefront.
constexpr int kBwdWaves = 4;
constexpr int kBwdChunk = 32;
constexpr int kBwdMaxGroups = 256;

static int backward_groups(int64_t n) {
  const int64_t chunks = (n + kBwdChunk - 1) / kBwdChunk;
  const int64_t g = (chunks + kBwdWaves - 1) / kBwdWaves;
  return (int)(g > kBwdMaxGroups ? kBwdMaxGroups : (g < 1 ? 1 : g));
}

static int backward_blocks(int64_t n) { return kBwdWaves * backward_groups(n); }

// Spatial bins of the latent-gradient scatter: squares of kBinTex (or a
// larger power of two, keeping at most kMaxBins bins) level-0 texels.
constexpr int kBinTex = 32;
constexpr int kMaxBins = 4096;
constexpr int kBinSamplesPerBlock = 4096;  // samples per workgroup of the count / scatter passes
constexpr int kBinWindowFloats = 12288;    // largest LDS of one bin's texel windows (48 KB)

// LDS (floats) for the texel windows of one bin: per level at most
// bin_tex W_k / W_0 + 4 texels along each axis (the range of positions plus
// one texel of margin below and two above), 3 channels, capped.
static int bin_window_floats(const LatArgs &lat, int bin_tex) {
  int64_t total = 0;
  for (int k = 0; k < lat.n_levels; ++k) {
    const int64_t nc = (int64_t)bin_tex * lat.lv[k].w / lat.lv[0].w + 4;
    const int64_t nr = (int64_t)bin_tex * lat.lv[k].h / lat.lv[0].h + 4;
    total += 3 * std::min<int64_t>(nc, lat.lv[k].w) * std::min<int64_t>(nr, lat.lv[k].h);
  }
  return (int)std::min<int64_t>(total, kBinWindowFloats);
}

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

BwdLayout backward_layout(const MlpShape &s, const LatArgs &lat, int64_t n) {
  BwdLayout L{};
  L.n_blocks = backward_blocks(n);
  L.n_params = n_params_of(s);
  L.n_feat = 3 * lat.n_levels;
  if (lat.address == 0 && n < ((int64_t)1 << 31)) {  // sample indices of the bins are int32
    int t = kBinTex;
    const int w = lat.lv[0].w, h = lat.lv[0].h;
    while ((int64_t)((w + t - 1) / t) * ((h + t - 1) / t) > kMaxBins) t *= 2;
    L.bin_tex = t;
    L.bins_x = (w + t - 1) / t;
    L.bins_y = (h + t - 1) / t;
    L.n_bins = L.bins_x * L.bins_y;
    L.bin_lds = bin_window_floats(lat, t);
  }
  size_t off = 0;
  L.wpart_off = off;
  off = align256(off + (size_t)L.n_blocks * L.n_params * sizeof(float));
  L.dx_off = off;
  off = align256(off + (size_t)n * L.n_feat * sizeof(float));
  L.count_off = off;
  off = align256(off + (size_t)L.n_bins * sizeof(int32_t));
  L.cursor_off = off;
  off = align256(off + (size_t)L.n_bins * sizeof(int32_t));
  L.perm_off = off;
  off = align256(off + (size_t)(L.n_bins ? n : 0) * sizeof(int32_t));
  L.total = off + 256;
  return L;
}

struct ReduceArgs {
  const float *part;
  int n_blocks;
  int n_params;
  int n_layers;
  int dims[kMaxLayers + 1];
  float *W[kMaxLayers];
  float *b[kMaxLayers];
};

// grad[p] = sum over workgroups of part[b][p], added in FP64, rounded once.
// A workgroup owns 64 consecutive parameters (one per lane, coalesced
// loads); its kReduceWaves wavefronts each add every kReduceWaves-th
// workgroup's partials, and the wavefront sums are then added in wavefront
// order, so the result does not depend on timing.
constexpr int kReduceWaves = 16;
__global__ __launch_bounds__(64 * kReduceWaves) void reduce_f64_kernel(ReduceArgs r) {
  __shared__ double wsum[kReduceWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (p < r.n_params) {
#pragma unroll 8
    for (int b = w; b < r.n_blocks; b += kReduceWaves) s += (double)r.part[(int64_t)b * r.n_params + p];
  }
  wsum[w][lane] = s;
  __syncthreads();
  if (w != 0 || p >= r.n_params) return;
  s = 0.0;
#pragma unroll
  for (int i = 0; i < kReduceWaves; ++i) s += wsum[i][lane];
  int off = p;
  for (int l = 0; l < r.n_layers; ++l) {
    const int nw = r.dims[l] * r.dims[l + 1];
    if (off < nw) {
      r.W[l][off] = (float)s;
      return;
    }
    off -= nw;
    if (off < r.dims[l + 1]) {
      r.b[l][off] = (float)s;
      return;
    }
    off -= r.dims[l + 1];
  }
}

// ---------------------------------------------------------------------------
// Pass 1 on the matrix cores (FP32 operands, v_mfma_f32_32x32x2f32)
//
// A wavefront takes 32 samples per step (the 32 columns of the matrix
// tiles). Every product is a 32 x 32 tile of units x samples: the weights
// are the A operand (row = output unit, one float per lane), the layer input
// the B operand. In the accumulator a lane holds rows 8 j + 4 h + r (j, r < 4,
// h = lane / 32) of sample lane % 32; K-step t of a product whose input is
// such a tile takes element t of it (lane half h supplying unit
// 8 (t / 4) + 4 h + t % 4 of the tile), so layers chain in registers in both
// directions and the ReLU mask of a delta is the activation at the same
// register. The first layer's K-slots hold per lane half two levels'
// features: slot 2 s + h is channel s % 3 of level 2 h + s / 3 (s < 6), u
// or v (s = 6), the constant 1 that carries the bias (s = 7, h = 0) or
// padding. Weight gradients contract over the samples: each step writes the
// deltas and the layer inputs transposed to LDS ([unit][sample], even
// samples first) and accumulates D A^T over 16 K-steps of two samples;
// bias gradients are row sums of the staged deltas.
// ---------------------------------------------------------------------------
typedef float bf32x16 __attribute__((ext_vector_type(16)));
typedef float bf32x4 __attribute__((ext_vector_type(4)));

constexpr int kStS = 36;  // row stride (floats) of the transposed staging

template <int MT, int NL>
struct BwdMap {
  static constexpr int HP = 32 * MT;        // padded hidden width
  static constexpr int S0 = 17;             // row stride of the first layer (16 K-slots)
  static constexpr int SH = HP + 1;         // row stride of the other layers
  static constexpr int NH = NL - 2;         // hidden-to-hidden layers
  static constexpr int oW0 = 0;
  static constexpr int oWh = oW0 + HP * S0;
  static constexpr int oWo = oWh + NH * HP * SH;
  static constexpr int oB = (oWo + 32 * SH + 3) & ~3;  // bias fragments [layer 1..NL-1][mt][h][16]
  static constexpr int nB = (NH * MT + 1) * 32;
  static constexpr int oStage = (oB + nB + 3) & ~3;
  static constexpr int stage_rows = HP + (HP > 32 ? HP : 32);
  static constexpr int stage = stage_rows * kStS;    // Dt then At, per wavefront
  static constexpr int total = oStage + kBwdWaves * stage;
  __device__ static int bias(int l, int mt) { return oB + ((l - 1) * MT + mt) * 32; }  // l = 1 .. NL - 1
};

// Unit of the previous layer's tile fed to K-step s by lane half h.
__device__ __forceinline__ int chain_unit(int s, int h) {
  return 32 * (s >> 4) + 8 * ((s & 15) >> 2) + 4 * h + (s & 3);
}

// Feature index of first-layer K-slot 2 s + h (-1: padding, -2: the bias).
__device__ __forceinline__ int slot_feature(int s, int h, int n_levels) {
  if (s < 6) {
    const int lvl = 2 * h + s / 3;
    return lvl < n_levels ? 3 * lvl + s % 3 : -1;
  }
  if (s == 6) return 3 * n_levels + h;
  return h == 0 ? -2 : -1;
}

__device__ __forceinline__ bf32x16 mfma32(float a, float b, bf32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <int MT, int NL>
__global__ __launch_bounds__(64 * kBwdWaves) __attribute__((amdgpu_waves_per_eu(1, 1)))
void backward_mfma_kernel(BackwardArgs a) {
  using M = BwdMap<MT, NL>;
  constexpr int HP = M::HP;
  extern __shared__ float bwd_lds[];
  float *lds = bwd_lds;
  const int tid = threadIdx.x;
  const int lane = tid & 63, h = lane >> 5, c32 = lane & 31;
  const int wave = tid >> 6;
  const int hid = a.dims[1], n_out = a.dims[NL], d0 = a.dims[0];
  const int n_levels = a.lat.n_levels;

  // ---- weights into LDS, zero-padded (every wavefront of the group shares them)
  for (int i = tid; i < HP * 16; i += 64 * kBwdWaves) {
    const int row = i >> 4, k = i & 15;
    const int f = slot_feature(k >> 1, k & 1, n_levels);
    float v = 0.0f;
    if (row < hid) v = f >= 0 ? a.W[0][row * d0 + f] : (f == -2 ? a.b[0][row] : 0.0f);
    lds[M::oW0 + row * M::S0 + k] = v;
  }
#pragma unroll
  for (int l = 1; l <= M::NH; ++l)
    for (int i = tid; i < HP * HP; i += 64 * kBwdWaves) {
      const int row = i / HP, col = i % HP;
      lds[M::oWh + (l - 1) * HP * M::SH + row * M::SH + col] = (row < hid && col < hid) ? a.W[l][row * hid + col] : 0.0f;
    }
  for (int i = tid; i < 32 * HP; i += 64 * kBwdWaves) {
    const int row = i / HP, col = i % HP;
    lds[M::oWo + row * M::SH + col] = (row < n_out && col < hid) ? a.W[NL - 1][row * hid + col] : 0.0f;
  }
  for (int i = tid; i < M::nB; i += 64 * kBwdWaves) {
    const int g = i / 32, e = i % 32;  // g = (l - 1) MT + mt, e = 16 h + 4 j + r
    const int l = g / MT + 1 < NL - 1 ? g / MT + 1 : NL - 1;
    const int mt = l == NL - 1 ? 0 : g % MT;
    const int row = 32 * mt + 8 * ((e & 15) >> 2) + 4 * (e >> 4) + (e & 3);
    const int rows = l == NL - 1 ? n_out : hid;
    lds[M::oB + i] = row < rows ? a.b[l][row] : 0.0f;
  }
  float *Dt = lds + M::oStage + wave * M::stage;
  float *At = Dt + HP * kStS;
  // the staging rows a layer input does not fill stay zero (first-layer K-slots 16..31)
  for (int i = lane; i < M::stage; i += 64) Dt[i] = 0.0f;
  __syncthreads();

  const float *W0s = lds + M::oW0;
  const float *Wo = lds + M::oWo;
  const bf32x16 zero = {};

  // weight-gradient accumulators: first layer [mt] (columns = K-slots), hidden
  // layers [l][mt][nt], output [nt]; bias gradients of rows `lane` (hidden)
  bf32x16 g0[MT], gh[M::NH > 0 ? M::NH : 1][MT][MT], go[MT];
  float gbh[M::NH > 0 ? M::NH : 1], gbo = 0.0f;
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    g0[i] = zero;
    go[i] = zero;
#pragma unroll
    for (int l = 0; l < (M::NH > 0 ? M::NH : 1); ++l)
#pragma unroll
      for (int j = 0; j < MT; ++j) gh[l][i][j] = zero;
  }
#pragma unroll
  for (int l = 0; l < (M::NH > 0 ? M::NH : 1); ++l) gbh[l] = 0.0f;

  // staging helpers: a tile in accumulator layout -> rows [row0, row0 + 32)
  // of a transposed buffer (column of sample n: 16 (n % 2) + n / 2)
  const int scol = 16 * (c32 & 1) + (c32 >> 1);
  auto stage_tile = [&](float *buf, int row0, const bf32x16 &t) {
#pragma unroll
    for (int i = 0; i < 16; ++i) buf[(row0 + 8 * (i >> 2) + 4 * h + (i & 3)) * kStS + scol] = t[i];
  };
  // the 16 K-step operands of row `row` (samples 2 s + h, s < 16)
  auto stage_row = [&](const float *buf, int row, float (&v)[16]) {
    const bf32x4 *p = reinterpret_cast<const bf32x4 *>(buf + row * kStS + 16 * h);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bf32x4 x = p[q];
      v[4 * q] = x[0];
      v[4 * q + 1] = x[1];
      v[4 * q + 2] = x[2];
      v[4 * q + 3] = x[3];
    }
  };
  // sum over the 32 samples of staged row `row`
  auto row_sum = [&](const float *buf, int row) {
    const bf32x4 *p = reinterpret_cast<const bf32x4 *>(buf + row * kStS);
    float sum = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bf32x4 x = p[q];
      sum += (x[0] + x[1]) + (x[2] + x[3]);
    }
    return sum;
  };
  // dW += Dt(MT_D tiles) At(NT_A tiles)^T over the 16 K-steps
  auto accum_dw = [&](auto &&acc, int mtn, int ntn) {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int mt = 0; mt < mtn; ++mt) {
      float av[16];
      stage_row(Dt, 32 * mt + c32, av);
#pragma unroll
      for (int nt = 0; nt < ntn; ++nt) {
        float bv[16];
        stage_row(At, 32 * nt + c32, bv);
#pragma unroll
        for (int q = 0; q < 16; ++q) acc(mt, nt) = mfma32(av[q], bv[q], acc(mt, nt));
      }
    }
    asm volatile("" ::: "memory");
  };

  const int64_t n_chunks = (a.n + kBwdChunk - 1) / kBwdChunk;
  const int64_t stride = (int64_t)gridDim.x * kBwdWaves;
  for (int64_t chunk = (int64_t)blockIdx.x * kBwdWaves + wave; chunk < n_chunks; chunk += stride) {
    const int64_t smp = chunk * kBwdChunk + c32;
    const bool valid = smp < a.n;
    const float2 uv = a.uv[valid ? smp : a.n - 1];

    // ---- features of this lane half's K-slots
    float x[8];
    {
      const float3 c0 = sample_f32(a.lat.lv[2 * h], uv.x, uv.y, a.lat.address);
      const float3 c1 = sample_f32(a.lat.lv[2 * h + 1], uv.x, uv.y, a.lat.address);
      x[0] = c0.x; x[1] = c0.y; x[2] = c0.z;
      x[3] = c1.x; x[4] = c1.y; x[5] = c1.z;
      x[6] = h ? uv.y : uv.x;
      x[7] = h ? 0.0f : 1.0f;
    }

    // ---- forward
    bf32x16 act[NL - 1][MT];  // ReLU outputs of the hidden layers
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      bf32x16 z = zero;
#pragma unroll
      for (int s = 0; s < 8; ++s) z = mfma32(W0s[(32 * mt + c32) * M::S0 + 2 * s + h], x[s], z);
#pragma unroll
      for (int i = 0; i < 16; ++i) z[i] = fmaxf(z[i], 0.0f);
      act[0][mt] = z;
    }
#pragma unroll
    for (int l = 1; l <= M::NH; ++l) {
      const float *Wl = lds + M::oWh + (l - 1) * HP * M::SH;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const bf32x4 *bp = reinterpret_cast<const bf32x4 *>(lds + M::bias(l, mt) + 16 * h);
        const bf32x4 b0 = bp[0], b1 = bp[1], b2 = bp[2], b3 = bp[3];
        bf32x16 z = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3],
                     b2[0], b2[1], b2[2], b2[3], b3[0], b3[1], b3[2], b3[3]};
#pragma unroll
        for (int s = 0; s < 16 * MT; ++s)
          z = mfma32(Wl[(32 * mt + c32) * M::SH + chain_unit(s, h)], act[l - 1][s >> 4][s & 15], z);
#pragma unroll
        for (int i = 0; i < 16; ++i) z[i] = fmaxf(z[i], 0.0f);
        act[l][mt] = z;
      }
    }
    bf32x16 dout;
    {
      const bf32x4 *bp = reinterpret_cast<const bf32x4 *>(lds + M::bias(NL - 1, 0) + 16 * h);
      const bf32x4 b0 = bp[0], b1 = bp[1];
      bf32x16 z = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3], 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 16 * MT; ++s)
        z = mfma32(Wo[c32 * M::SH + chain_unit(s, h)], act[NL - 2][s >> 4][s & 15], z);
      // output deltas: g f (1 - f) on rows 8 j + 4 h + r < n_out (j < 2)
      dout = zero;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int row = 8 * (i >> 2) + 4 * h + (i & 3);
        if (row < n_out && valid) {
          const float f = 1.0f / (1.0f + expf(-z[i]));
          dout[i] = a.grad_out[smp * n_out + row] * f * (1.0f - f);
        }
      }
    }

    // ---- output layer: weight and bias gradients, delta of the last hidden layer
    stage_tile(Dt, 0, dout);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) stage_tile(At, 32 * mt, act[NL - 2][mt]);
    accum_dw([&](int, int nt) -> bf32x16 & { return go[nt]; }, 1, MT);
    if (lane < 16) gbo += row_sum(Dt, lane);
    bf32x16 del[MT];
    {
      const int tk = n_out > 8 ? 8 : 4;  // K-steps covering rows 0 .. n_out - 1
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        bf32x16 z = zero;
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (t < tk) z = mfma32(Wo[(8 * (t >> 2) + 4 * h + (t & 3)) * M::SH + 32 * mt + c32], dout[t], z);
#pragma unroll
        for (int i = 0; i < 16; ++i) del[mt][i] = act[NL - 2][mt][i] > 0.0f ? z[i] : 0.0f;
      }
    }
    // ---- hidden layers, top down
#pragma unroll
    for (int l = M::NH; l >= 1; --l) {
      const float *Wl = lds + M::oWh + (l - 1) * HP * M::SH;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        stage_tile(Dt, 32 * mt, del[mt]);
        stage_tile(At, 32 * mt, act[l - 1][mt]);
      }
      accum_dw([&](int mt, int nt) -> bf32x16 & { return gh[l - 1][mt][nt]; }, MT, MT);
      if (lane < HP) gbh[l - 1] += row_sum(Dt, lane);
      bf32x16 nd[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        bf32x16 z = zero;
#pragma unroll
        for (int s = 0; s < 16 * MT; ++s)
          z = mfma32(Wl[chain_unit(s, h) * M::SH + 32 * mt + c32], del[s >> 4][s & 15], z);
#pragma unroll
        for (int i = 0; i < 16; ++i) nd[mt][i] = act[l - 1][mt][i] > 0.0f ? z[i] : 0.0f;
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) del[mt] = nd[mt];
    }
    // ---- first layer: weight gradients over the K-slots (slot 14 = bias)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) stage_tile(Dt, 32 * mt, del[mt]);
#pragma unroll
    for (int s = 0; s < 8; ++s) At[(2 * s + h) * kStS + scol] = x[s];
    accum_dw([&](int mt, int) -> bf32x16 & { return g0[mt]; }, MT, 1);
    // ---- feature gradient dx = W0^T D0: rows = latent features
    {
      const int f = c32;  // feature of A-operand row c32
      const int lvl = f / 3;
      const int slot = (lvl < n_levels && f < 12) ? 2 * (3 * (lvl & 1) + f % 3) + (lvl >> 1) : -1;
      bf32x16 z = zero;
#pragma unroll
      for (int s = 0; s < 16 * MT; ++s) {
        const float w = slot >= 0 ? W0s[chain_unit(s, h) * M::S0 + slot] : 0.0f;
        z = mfma32(w, del[s >> 4][s & 15], z);
      }
      if (valid) {
        float *out = a.dx + smp * a.n_feat;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int row = 8 * (i >> 2) + 4 * h + (i & 3);
          if (row < a.n_feat) out[row] = z[i];
        }
      }
    }
  }

  // ---- this wavefront's partial sums (parameters in unpadded order)
  float *part = a.wpart + ((int64_t)blockIdx.x * kBwdWaves + wave) * a.n_params;
  int off = 0;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 32 * mt + 8 * (i >> 2) + 4 * h + (i & 3);
      const int k = c32;
      if (row < hid && k < 16) {
        const int f = slot_feature(k >> 1, k & 1, n_levels);
        if (f >= 0) part[off + row * d0 + f] = g0[mt][i];
        if (f == -2) part[off + hid * d0 + row] = g0[mt][i];
      }
    }
  off += hid * d0 + hid;
#pragma unroll
  for (int l = 0; l < M::NH; ++l) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < MT; ++nt)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int row = 32 * mt + 8 * (i >> 2) + 4 * h + (i & 3), col = 32 * nt + c32;
          if (row < hid && col < hid) part[off + row * hid + col] = gh[l][mt][nt][i];
        }
    if (lane < hid) part[off + hid * hid + lane] = gbh[l];
    off += hid * hid + hid;
  }
#pragma unroll
  for (int nt = 0; nt < MT; ++nt)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 8 * (i >> 2) + 4 * h + (i & 3), col = 32 * nt + c32;
      if (row < n_out && col < hid) part[off + row * hid + col] = go[nt][i];
    }
  if (lane < n_out) part[off + n_out * hid + lane] = gbo;
}

// ---------------------------------------------------------------------------
// Pass 2: latent gradients
// ---------------------------------------------------------------------------

// Bin of a sample: the square of level-0 texels holding its clamped level-0
// sampling position.
__device__ __forceinline__ int bin_of(const BackwardArgs &a, float2 uv) {
  const LevelArgs &L = a.lat.lv[0];
  float x = fmaf(uv.x, L.fw, -0.5f) + L.sx;
  float y = fmaf(uv.y, L.fh, -0.5f) + L.sy;
  x = fminf(fmaxf(x, 0.0f), L.fw - 1.0f);  // NaN becomes 0
  y = fminf(fmaxf(y, 0.0f), L.fh - 1.0f);
  const int bx = min((int)x / a.bin_tex, a.bins_x - 1);
  const int by = min((int)y / a.bin_tex, a.bins_y - 1);
  return by * a.bins_x + bx;
}

// Per-bin sample counts: a histogram in LDS per workgroup, added to the
// global counts (which start at zero).
__global__ __launch_bounds__(256) void bin_count_kernel(BackwardArgs a) {
  extern __shared__ int32_t hist[];
  for (int k = threadIdx.x; k < a.n_bins; k += 256) hist[k] = 0;
  __syncthreads();
  const int64_t s0 = (int64_t)blockIdx.x * kBinSamplesPerBlock;
  for (int i = threadIdx.x; i < kBinSamplesPerBlock; i += 256) {
    const int64_t s = s0 + i;
    if (s < a.n) atomicAdd(&hist[bin_of(a, a.uv[s])], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < a.n_bins; k += 256)
    if (hist[k]) atomicAdd(&a.bin_count[k], hist[k]);
}

// Exclusive prefix sum of the counts, in place; the cursors start at the
// same offsets. One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void bin_scan_kernel(BackwardArgs a) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int per = (a.n_bins + 1023) / 1024;
  const int k0 = t * per, k1 = min(k0 + per, a.n_bins);
  int32_t sum = 0;
  for (int k = k0; k < k1; ++k) sum += a.bin_count[k];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int32_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = part[t] - sum;
  for (int k = k0; k < k1; ++k) {
    const int32_t c = a.bin_count[k];
    a.bin_count[k] = run;
    a.bin_cursor[k] = run;
    run += c;
  }
}

// Sample indices grouped by bin: each workgroup ranks its samples per bin in
// LDS, reserves a range per bin with one global atomic, then writes. The
// order inside a bin depends on timing (as does the order of the atomics
// that follow it).
__global__ __launch_bounds__(256) void bin_scatter_kernel(BackwardArgs a) {
  extern __shared__ int32_t lds[];
  int32_t *local = lds, *base = lds + a.n_bins;
  for (int k = threadIdx.x; k < a.n_bins; k += 256) local[k] = 0;
  __syncthreads();
  constexpr int kPer = kBinSamplesPerBlock / 256;
  const int64_t s0 = (int64_t)blockIdx.x * kBinSamplesPerBlock;
  int key[kPer], rank[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int64_t s = s0 + threadIdx.x + 256 * i;
    key[i] = s < a.n ? bin_of(a, a.uv[s]) : -1;
    rank[i] = key[i] >= 0 ? atomicAdd(&local[key[i]], 1) : 0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < a.n_bins; k += 256)
    if (local[k]) base[k] = atomicAdd(&a.bin_cursor[k], local[k]);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kPer; ++i)
    if (key[i] >= 0) a.perm[base[key[i]] + rank[i]] = (int32_t)(s0 + threadIdx.x + 256 * i);
}

// Texel window of one level reachable from one bin: columns [c0, c0 + nc),
// rows [r0, r0 + nr); lds: offset in floats, or -1 when the window does not
// fit the workgroup's LDS (that level's taps then go to global atomics).
struct BinWindow {
  int c0, nc, r0, nr, lds;
};

// Texel range along one axis of level k reached by level-0 positions in
// [p_lo, p_hi): the position maps linearly between levels; one texel of
// margin on each side absorbs rounding (a tap outside the range still takes
// the global path, so the range need not be exact).
__device__ __forceinline__ void window_axis(float p_lo, float p_hi, bool open_lo, bool open_hi, float f0, float s0,
                                            float fk, float sk, int n, int &c0, int &nc) {
  const float q = fk / f0;
  const float x_lo = (p_lo + 0.5f - s0) * q - 0.5f + sk;
  const float x_hi = (p_hi + 0.5f - s0) * q - 0.5f + sk;
  int lo = open_lo ? 0 : (int)floorf(fminf(fmaxf(x_lo, 0.0f), (float)(n - 1))) - 1;
  int hi = open_hi ? n - 1 : (int)floorf(fminf(fmaxf(x_hi, 0.0f), (float)(n - 1))) + 2;
  lo = max(lo, 0);
  hi = min(hi, n - 1);
  c0 = lo;
  nc = hi - lo + 1;
}

// Sub-bin of a sample inside its bin: 8 x 8 squares of bin_tex / 8 level-0
// texels (the same clamped position as bin_of).
__device__ __forceinline__ int sub_of(const BackwardArgs &a, float2 uv, int bx, int by) {
  const LevelArgs &L = a.lat.lv[0];
  float x = fmaf(uv.x, L.fw, -0.5f) + L.sx;
  float y = fmaf(uv.y, L.fh, -0.5f) + L.sy;
  x = fminf(fmaxf(x, 0.0f), L.fw - 1.0f);
  y = fminf(fmaxf(y, 0.0f), L.fh - 1.0f);
  const int st = a.bin_tex >> 3;
  const int sx = min(((int)x - bx * a.bin_tex) / st, 7), sy = min(((int)y - by * a.bin_tex) / st, 7);
  return 8 * max(sy, 0) + max(sx, 0);
}

// Bilinear-tap gradients of one level, accumulated while consecutive samples
// keep the same taps (a lane walks the samples of one sub-bin, which share
// the taps of the coarse levels most of the time) and added to the LDS
// window (or, outside it, to the gradient texture) when they change.
struct TapCache {
  int ix, iy;      // unclamped left / top tap of the cached contributions
  float g[4][3];   // per tap, per channel
};

__device__ __forceinline__ void cache_flush(TapCache &c, const BackwardArgs &a, int k, const BinWindow &wk,
                                            float *win) {
  if (c.ix == INT_MIN) return;
  const LevelArgs &L = a.lat.lv[k];
  const int i0 = address_coord(c.ix, L.w, 0), i1 = address_coord(c.ix + 1, L.w, 0);
  const int j0 = address_coord(c.iy, L.h, 0), j1 = address_coord(c.iy + 1, L.h, 0);
  const int ii[4] = {i0, i1, i0, i1};
  const int jj[4] = {j0, j0, j1, j1};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int col = ii[q] - wk.c0, row = jj[q] - wk.r0;
    if (wk.lds >= 0 && (unsigned)col < (unsigned)wk.nc && (unsigned)row < (unsigned)wk.nr) {
      float *p = win + wk.lds + 3 * (row * wk.nc + col);
      atomicAdd(p + 0, c.g[q][0]);
      atomicAdd(p + 1, c.g[q][1]);
      atomicAdd(p + 2, c.g[q][2]);
    } else {
      float *p = a.grad_lat[k] + ((int64_t)jj[q] * L.w + ii[q]) * 3;
      unsafeAtomicAdd(p + 0, c.g[q][0]);
      unsafeAtomicAdd(p + 1, c.g[q][1]);
      unsafeAtomicAdd(p + 2, c.g[q][2]);
    }
  }
  c.ix = INT_MIN;
}

// One bin per workgroup. The bin's samples are sorted by sub-bin in LDS (in
// rounds of kBinChunk); thread t then walks the samples of sub-bin t % 64
// with stride 4 (t / 64 the phase), so the 64 lanes of a wavefront work in
// 64 different places of the bin and each lane's consecutive samples are
// neighbours. LDS: the texel windows (bin_lds floats), then the sorted
// sample indices and the sub-bin counts.
constexpr int kBinChunk = 2048;
constexpr int kSubBins = 64;

__global__ __launch_bounds__(256) void bin_accum_kernel(BackwardArgs a) {
  extern __shared__ float win[];
  int32_t *sorted = reinterpret_cast<int32_t *>(win + a.bin_lds);
  int32_t *sub_start = sorted + kBinChunk;      // [kSubBins + 1]
  int32_t *sub_cursor = sub_start + kSubBins + 1;  // [kSubBins]
  const int bin = blockIdx.x;
  const int start = a.bin_count[bin];
  const int end = bin + 1 < a.n_bins ? a.bin_count[bin + 1] : (int)a.n;
  if (start >= end) return;
  const int bx = bin % a.bins_x, by = bin / a.bins_x;
  const int n_levels = a.lat.n_levels;
  const int tid = threadIdx.x;
  BinWindow wk[kMaxLevels];
  int used = 0;
  const LevelArgs &L0 = a.lat.lv[0];
#pragma unroll
  for (int k = 0; k < kMaxLevels; ++k) {
    wk[k].lds = -1;
    wk[k].c0 = wk[k].r0 = wk[k].nc = wk[k].nr = 0;
    if (k < n_levels) {
      const LevelArgs &L = a.lat.lv[k];
      window_axis((float)(bx * a.bin_tex), (float)((bx + 1) * a.bin_tex), bx == 0, bx == a.bins_x - 1, L0.fw, L0.sx,
                  L.fw, L.sx, L.w, wk[k].c0, wk[k].nc);
      window_axis((float)(by * a.bin_tex), (float)((by + 1) * a.bin_tex), by == 0, by == a.bins_y - 1, L0.fh, L0.sy,
                  L.fh, L.sy, L.h, wk[k].r0, wk[k].nr);
      const int sz = 3 * wk[k].nc * wk[k].nr;
      if (used + sz <= a.bin_lds) {
        wk[k].lds = used;
        used += sz;
      }
    }
  }
  for (int i = tid; i < used; i += 256) win[i] = 0.0f;
  const int sub = tid & (kSubBins - 1), phase = tid >> 6;
  for (int c0 = start; c0 < end; c0 += kBinChunk) {
    const int m = min(kBinChunk, end - c0);
    // counting sort of this round's samples by sub-bin
    if (tid <= kSubBins) sub_start[tid] = 0;
    __syncthreads();
    for (int i = tid; i < m; i += 256) atomicAdd(&sub_start[1 + sub_of(a, a.uv[a.perm[c0 + i]], bx, by)], 1);
    __syncthreads();
    if (tid < 64) {  // inclusive scan of the 64 counts (one wavefront)
      int v = sub_start[1 + tid];
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (tid >= o) v += t;
      }
      sub_start[1 + tid] = v;
    }
    __syncthreads();
    if (tid < kSubBins) sub_cursor[tid] = sub_start[tid];
    __syncthreads();
    for (int i = tid; i < m; i += 256) {
      const int s = a.perm[c0 + i];
      const int key = sub_of(a, a.uv[s], bx, by);
      sorted[atomicAdd(&sub_cursor[key], 1)] = s;
    }
    __syncthreads();
    // this thread's samples: sub-bin `sub`, every fourth
    TapCache cache[kMaxLevels];
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) cache[k].ix = INT_MIN;
    const int j1 = sub_start[sub + 1];
    for (int j = sub_start[sub] + phase; j < j1; j += 4) {
      const int s = sorted[j];
      const float2 uv = a.uv[s];
      const float *g = a.dx + (int64_t)s * a.n_feat;
#pragma unroll
      for (int k = 0; k < kMaxLevels; ++k) {
        if (k < n_levels) {
          const LevelArgs &L = a.lat.lv[k];
          float x = fmaf(uv.x, L.fw, -0.5f) + L.sx;
          float y = fmaf(uv.y, L.fh, -0.5f) + L.sy;
          x = fminf(fmaxf(x, -16777216.0f), 16777216.0f);
          y = fminf(fmaxf(y, -16777216.0f), 16777216.0f);
          const float xf = floorf(x), yf = floorf(y);
          const float fx = x - xf, fy = y - yf;
          const int ix = (int)xf, iy = (int)yf;
          if (ix != cache[k].ix || iy != cache[k].iy) {
            cache_flush(cache[k], a, k, wk[k], win);
            cache[k].ix = ix;
            cache[k].iy = iy;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int ch = 0; ch < 3; ++ch) cache[k].g[q][ch] = 0.0f;
          }
          const float gx = 1.0f - fx, gy = 1.0f - fy;
          const float w[4] = {gx * gy, fx * gy, gx * fy, fx * fy};
          const float d[3] = {g[3 * k], g[3 * k + 1], g[3 * k + 2]};
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) cache[k].g[q][ch] = fmaf(w[q], d[ch], cache[k].g[q][ch]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k)
      if (k < n_levels) cache_flush(cache[k], a, k, wk[k], win);
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kMaxLevels; ++k) {
    if (k < n_levels && wk[k].lds >= 0) {
      const int nc = wk[k].nc, cnt = 3 * nc * wk[k].nr;
      float *G = a.grad_lat[k];
      const int w = a.lat.lv[k].w;
      for (int i = tid; i < cnt; i += 256) {
        const float v = win[wk[k].lds + i];
        if (v != 0.0f) {
          const int texel = i / 3, ch = i - 3 * texel;
          const int r = texel / nc, c = texel - r * nc;
          unsafeAtomicAdd(G + ((int64_t)(wk[k].r0 + r) * w + wk[k].c0 + c) * 3 + ch, v);
        }
      }
    }
  }
}

// Wrap addressing: every tap of every sample is a global atomic.
__global__ __launch_bounds__(256) void scatter_direct_kernel(BackwardArgs a) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= a.n) return;
  const float2 uv = a.uv[s];
  const float *g = a.dx + s * a.n_feat;
#pragma unroll
  for (int k = 0; k < kMaxLevels; ++k) {
    if (k < a.lat.n_levels) {
      const LevelArgs &L = a.lat.lv[k];
      const Taps t = tap_coords(uv.x, uv.y, L, a.lat.address);
      const float gx = 1.0f - t.fx, gy = 1.0f - t.fy;
      const float w[4] = {gx * gy, t.fx * gy, gx * t.fy, t.fx * t.fy};
      const int ii[4] = {t.i0, t.i1, t.i0, t.i1};
      const int jj[4] = {t.j0, t.j0, t.j1, t.j1};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float *p = a.grad_lat[k] + ((int64_t)jj[q] * L.w + ii[q]) * 3;
        unsafeAtomicAdd(p + 0, w[q] * g[3 * k]);
        unsafeAtomicAdd(p + 1, w[q] * g[3 * k + 1]);
        unsafeAtomicAdd(p + 2, w[q] * g[3 * k + 2]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Forward decode of continuous (float) latents on the FP32 matrix cores: the
// forward half of backward_mfma_kernel (same LDS weight layout, same
// 32-sample steps), ending in the sigmoid and the store. Weights come from
// the packed FP32 image (per layer W [rows_pad][cols_pad], then b).
// ---------------------------------------------------------------------------
template <int MT, int NL>
__global__ __launch_bounds__(64 * kBwdWaves) void forward_mfma_kernel(DecodeArgs a) {
  using M = BwdMap<MT, NL>;
  constexpr int HP = M::HP;
  extern __shared__ float fwd_lds[];
  float *lds = fwd_lds;
  const int tid = threadIdx.x;
  const int lane = tid & 63, h = lane >> 5, c32 = lane & 31;
  const int wave = tid >> 6;
  const PackLayout &L = a.lay;
  const int n_out = a.n_out, n_levels = a.lat.n_levels;
  const float *W0 = reinterpret_cast<const float *>(a.packed + L.w_off[0]);
  const float *B0 = reinterpret_cast<const float *>(a.packed + L.b_off[0]);
  const int hid = L.rows_pad[0] < HP ? L.rows_pad[0] : HP;  // padded rows hold zero weights

  for (int i = tid; i < HP * 16; i += 64 * kBwdWaves) {
    const int row = i >> 4, k = i & 15;
    const int f = slot_feature(k >> 1, k & 1, n_levels);
    float v = 0.0f;
    if (row < hid) v = f >= 0 ? W0[row * L.cols_pad[0] + f] : (f == -2 ? B0[row] : 0.0f);
    lds[M::oW0 + row * M::S0 + k] = v;
  }
#pragma unroll
  for (int l = 1; l <= M::NH; ++l) {
    const float *Wl = reinterpret_cast<const float *>(a.packed + L.w_off[l]);
    for (int i = tid; i < HP * HP; i += 64 * kBwdWaves) {
      const int row = i / HP, col = i % HP;
      lds[M::oWh + (l - 1) * HP * M::SH + row * M::SH + col] =
          (row < L.rows_pad[l] && col < L.cols_pad[l]) ? Wl[row * L.cols_pad[l] + col] : 0.0f;
    }
  }
  {
    const float *Wo = reinterpret_cast<const float *>(a.packed + L.w_off[NL - 1]);
    for (int i = tid; i < 32 * HP; i += 64 * kBwdWaves) {
      const int row = i / HP, col = i % HP;
      lds[M::oWo + row * M::SH + col] =
          (row < L.rows_pad[NL - 1] && col < L.cols_pad[NL - 1]) ? Wo[row * L.cols_pad[NL - 1] + col] : 0.0f;
    }
  }
  for (int i = tid; i < M::nB; i += 64 * kBwdWaves) {
    const int g = i / 32, e = i % 32;  // g = (l - 1) MT + mt, e = 16 h + 4 j + r
    const int l = g / MT + 1 < NL - 1 ? g / MT + 1 : NL - 1;
    const int mt = l == NL - 1 ? 0 : g % MT;
    const int row = 32 * mt + 8 * ((e & 15) >> 2) + 4 * (e >> 4) + (e & 3);
    const float *Bl = reinterpret_cast<const float *>(a.packed + L.b_off[l]);
    lds[M::oB + i] = row < L.rows_pad[l] ? Bl[row] : 0.0f;
  }
  __syncthreads();

  const float *W0s = lds + M::oW0;
  const float *Wos = lds + M::oWo;
  const bf32x16 zero = {};
  const int64_t n_chunks = (a.n + kBwdChunk - 1) / kBwdChunk;
  const int64_t stride = (int64_t)gridDim.x * kBwdWaves;
  for (int64_t chunk = (int64_t)blockIdx.x * kBwdWaves + wave; chunk < n_chunks; chunk += stride) {
    const int64_t smp = chunk * kBwdChunk + c32;
    const bool valid = smp < a.n;
    const float2 uv = a.uv[valid ? smp : a.n - 1];
    float x[8];
    {
      const float3 c0 = sample_f32(a.lat.lv[2 * h], uv.x, uv.y, a.lat.address);
      const float3 c1 = sample_f32(a.lat.lv[2 * h + 1], uv.x, uv.y, a.lat.address);
      x[0] = c0.x; x[1] = c0.y; x[2] = c0.z;
      x[3] = c1.x; x[4] = c1.y; x[5] = c1.z;
      x[6] = h ? uv.y : uv.x;
      x[7] = h ? 0.0f : 1.0f;
    }
    bf32x16 act[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      bf32x16 z = zero;
#pragma unroll
      for (int s = 0; s < 8; ++s) z = mfma32(W0s[(32 * mt + c32) * M::S0 + 2 * s + h], x[s], z);
#pragma unroll
      for (int i = 0; i < 16; ++i) z[i] = fmaxf(z[i], 0.0f);
      act[mt] = z;
    }
#pragma unroll
    for (int l = 1; l <= M::NH; ++l) {
      const float *Wl = lds + M::oWh + (l - 1) * HP * M::SH;
      bf32x16 nx[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const bf32x4 *bp = reinterpret_cast<const bf32x4 *>(lds + M::bias(l, mt) + 16 * h);
        const bf32x4 b0 = bp[0], b1 = bp[1], b2 = bp[2], b3 = bp[3];
        bf32x16 z = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3],
                     b2[0], b2[1], b2[2], b2[3], b3[0], b3[1], b3[2], b3[3]};
#pragma unroll
        for (int s = 0; s < 16 * MT; ++s)
          z = mfma32(Wl[(32 * mt + c32) * M::SH + chain_unit(s, h)], act[s >> 4][s & 15], z);
#pragma unroll
        for (int i = 0; i < 16; ++i) z[i] = fmaxf(z[i], 0.0f);
        nx[mt] = z;
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) act[mt] = nx[mt];
    }
    const bf32x4 *bp = reinterpret_cast<const bf32x4 *>(lds + M::bias(NL - 1, 0) + 16 * h);
    const bf32x4 b0 = bp[0], b1 = bp[1];
    bf32x16 z = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3], 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 16 * MT; ++s) z = mfma32(Wos[c32 * M::SH + chain_unit(s, h)], act[s >> 4][s & 15], z);
    if (valid) {
      // rows 8 j + 4 h + r (j < 2, r < 4) of this lane's sample
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int row0 = 8 * j + 4 * h;
        if (row0 >= n_out) continue;
        float f[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) f[r] = 1.0f / (1.0f + expf(-z[4 * j + r]));
        if (a.out_f16) {
          _Float16 *o = reinterpret_cast<_Float16 *>(a.out) + smp * n_out + row0;
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (row0 + r < n_out) o[r] = (_Float16)f[r];
        } else {
          float *o = reinterpret_cast<float *>(a.out) + smp * n_out + row0;
          if ((n_out & 3) == 0) {
            *reinterpret_cast<float4 *>(o) = make_float4(f[0], f[1], f[2], f[3]);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (row0 + r < n_out) o[r] = f[r];
          }
        }
      }
    }
  }
}

hipError_t launch_forward_f32(const DecodeArgs &a, const MlpShape &s, hipStream_t st) {
  const int groups = backward_groups(a.n);
  auto go = [&](auto kernel, size_t floats) {
    hipLaunchKernelGGL(kernel, dim3(groups), dim3(64 * kBwdWaves), floats * sizeof(float), st, a);
    return hipGetLastError();
  };
  const int mt = s.hid > 32 ? 2 : 1;
  if (mt == 1) {
    switch (s.n_layers) {
      case 2: return go(forward_mfma_kernel<1, 2>, BwdMap<1, 2>::oStage);
      case 3: return go(forward_mfma_kernel<1, 3>, BwdMap<1, 3>::oStage);
      case 4: return go(forward_mfma_kernel<1, 4>, BwdMap<1, 4>::oStage);
      default: return hipErrorInvalidValue;
    }
  }
  switch (s.n_layers) {
    case 2: return go(forward_mfma_kernel<2, 2>, BwdMap<2, 2>::oStage);
    case 3: return go(forward_mfma_kernel<2, 3>, BwdMap<2, 3>::oStage);
    case 4: return go(forward_mfma_kernel<2, 4>, BwdMap<2, 4>::oStage);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_backward(const BackwardArgs &a, const MlpShape &s, float *const *grad_W, float *const *grad_b,
                           hipStream_t st) {
  // latent gradients start at zero (fill kernel: no memset nodes in graphs)
  for (int k = 0; k < a.lat.n_levels; ++k) {
    hipError_t e = launch_fill_f32(a.grad_lat[k], (int64_t)a.lat.lv[k].w * a.lat.lv[k].h * 3, 0.0f, st);
    if (e != hipSuccess) return e;
  }
  hipError_t e;
  {
    const int groups = a.n_blocks / kBwdWaves;
    auto go = [&](auto kernel, size_t floats) {
      hipLaunchKernelGGL(kernel, dim3(groups), dim3(64 * kBwdWaves), floats * sizeof(float), st, a);
      return hipGetLastError();
    };
    const int mt = s.hid > 32 ? 2 : 1;
    if (mt == 1) {
      switch (s.n_layers) {
        case 2: e = go(backward_mfma_kernel<1, 2>, BwdMap<1, 2>::total); break;
        case 3: e = go(backward_mfma_kernel<1, 3>, BwdMap<1, 3>::total); break;
        case 4: e = go(backward_mfma_kernel<1, 4>, BwdMap<1, 4>::total); break;
        default: return hipErrorInvalidValue;
      }
    } else {
      switch (s.n_layers) {
        case 2: e = go(backward_mfma_kernel<2, 2>, BwdMap<2, 2>::total); break;
        case 3: e = go(backward_mfma_kernel<2, 3>, BwdMap<2, 3>::total); break;
        case 4: e = go(backward_mfma_kernel<2, 4>, BwdMap<2, 4>::total); break;
        default: return hipErrorInvalidValue;
      }
    }
  }
  if (e != hipSuccess) return e;
  ReduceArgs r;
  r.part = a.wpart;
  r.n_blocks = a.n_blocks;
  r.n_params = a.n_params;
  r.n_layers = s.n_layers;
  for (int l = 0; l <= s.n_layers; ++l) r.dims[l] = a.dims[l];
  for (int l = 0; l < s.n_layers; ++l) {
    r.W[l] = grad_W[l];
    r.b[l] = grad_b[l];
  }
  hipLaunchKernelGGL(reduce_f64_kernel, dim3((a.n_params + 63) / 64), dim3(64 * kReduceWaves), 0, st, r);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // latent gradients from dx
  if (a.n_bins == 0) {
    hipLaunchKernelGGL(scatter_direct_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
  }
  if ((e = launch_fill_f32(reinterpret_cast<float *>(a.bin_count), a.n_bins, 0.0f, st)) != hipSuccess) return e;
  const unsigned grid = (unsigned)((a.n + kBinSamplesPerBlock - 1) / kBinSamplesPerBlock);
  hipLaunchKernelGGL(bin_count_kernel, dim3(grid), dim3(256), a.n_bins * sizeof(int32_t), st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bin_scan_kernel, dim3(1), dim3(1024), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bin_scatter_kernel, dim3(grid), dim3(256), 2 * a.n_bins * sizeof(int32_t), st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bin_accum_kernel, dim3(a.n_bins), dim3(256),
                     (size_t)a.bin_lds * sizeof(float) + (kBinChunk + 2 * kSubBins + 1) * sizeof(int32_t), st, a);
  return hipGetLastError();
}

}  // namespace ntc
