// Backward of the FP32 decode for continuous latents (Sec. 3.2: gradients
// flow through the MLP into every latent element).
//
// One wavefront owns a chunk of 64 samples at a time (one sample per lane):
//   1. forward in registers (features, every layer input A_l),
//   2. D_{L-1} = g * f (1 - f); for l = L-1 .. 0:
//        the wave writes D_l and A_l of its 64 samples to LDS and the lanes
//        then add the 64-sample outer-product sum D_l^T A_l (and the column
//        sums for the bias) to the workgroup's FP32 accumulators in LDS,
//        each lane owning an (M/8) x (K/8) block of W_l;
//        D_{l-1} = (W_l^T D_l) * [A_l > 0]   (ReLU derivative 0 at 0);
//   3. dx = W_0^T D_0 is spread onto the four bilinear taps of every level
//      with FP32 atomics.
// Activations are recomputed per chunk, never stored in global memory. At
// the end every workgroup writes its FP32 partial sums; a second kernel adds
// the partials of all workgroups in FP64 and rounds once to FP32.
#include <hip/hip_runtime.h>

#include "ntc_device.hpp"
#include "ntc_internal.hpp"

namespace ntc {

// Persistent workgroups of the backward (two per compute unit of a 256-CU
// part; fewer for small batches). Depends on n only, so the workspace size
// is known on the host without a device query.
constexpr int kBwdMaxBlocks = 1024;
// Samples staged in LDS per round of the dW accumulation (a chunk of 64 takes
// 64 / kBwdStage rounds): with 16, a workgroup needs under 40 KB of LDS and
// four fit on a compute unit, one per SIMD.
constexpr int kBwdStage = 16;

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

size_t backward_workspace_bytes(const MlpShape &s, int n_blocks) {
  return (size_t)n_blocks * (size_t)n_params_of(s) * sizeof(float) + 256;
}

int backward_blocks(int64_t n) {
  const int64_t chunks = (n + 63) / 64;
  return (int)(chunks > kBwdMaxBlocks ? kBwdMaxBlocks : (chunks < 1 ? 1 : chunks));
}

// Padded widths used inside the kernel: inputs of layer 0 to 16, outputs of
// the last layer to 16.
template <int HID, int NL>
struct BwdDims {
  static constexpr int in(int l) { return l == 0 ? 16 : HID; }
  static constexpr int out(int l) { return l == NL - 1 ? 16 : HID; }
};

// Accumulate D^T A over the kBwdStage staged samples into acc (row-major
// [M][K] weights of the padded layer) and column sums of D into accb [M].
// Lane (a, b) = (lane / 8, lane % 8) owns rows [a BM, a BM + BM) and columns
// [b BK, b BK + BK) with BM = M / 8, BK = K / 8.
template <int M, int K>
__device__ __forceinline__ void accum_outer(const float *D, int ds, const float *A, int as, float *acc, float *accb,
                                            int lane) {
  constexpr int BM = M / 8, BK = K / 8;
  const int a = lane >> 3, b = lane & 7;
  float w[BM][BK];
  float bs[BM];
#pragma unroll
  for (int i = 0; i < BM; ++i) {
    bs[i] = 0.f;
#pragma unroll
    for (int j = 0; j < BK; ++j) w[i][j] = 0.f;
  }
  for (int s = 0; s < kBwdStage; ++s) {
    float dv[BM], av[BK];
#pragma unroll
    for (int i = 0; i < BM; ++i) dv[i] = D[s * ds + a * BM + i];
#pragma unroll
    for (int j = 0; j < BK; ++j) av[j] = A[s * as + b * BK + j];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
      bs[i] += dv[i];
#pragma unroll
      for (int j = 0; j < BK; ++j) w[i][j] = fmaf(dv[i], av[j], w[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < BM; ++i) {
#pragma unroll
    for (int j = 0; j < BK; ++j) acc[(a * BM + i) * K + b * BK + j] += w[i][j];
    if (b == 0) accb[a * BM + i] += bs[i];
  }
}

// Weights and biases of the layers, each as its own read-only, non-aliasing
// kernel argument: their loads are uniform and no store of the kernel can
// reach them, so the compiler reads them through the scalar cache once per
// wavefront instead of once per lane.
template <int HID, int NL>
__global__ __launch_bounds__(64) void backward_kernel(BackwardArgs a, const float *__restrict__ W0,
                                                      const float *__restrict__ W1, const float *__restrict__ W2,
                                                      const float *__restrict__ W3, const float *__restrict__ b0,
                                                      const float *__restrict__ b1, const float *__restrict__ b2,
                                                      const float *__restrict__ b3) {
  // Layer l's parameters (l is a constant wherever this is called), offset
  // by a zero the compiler cannot see through: `salt` differs per chunk and
  // per use, so the scalar loads of the weights stay where they are used
  // instead of being hoisted out of the chunk loop or shared between the
  // forward and the backward (thousands of weights held in scalar registers
  // would spill into vector lanes).
  auto Wl = [&](int l, int salt) {
    return (l == 0 ? W0 : (l == 1 ? W1 : (l == 2 ? W2 : W3))) + opaque_zero(salt);
  };
  auto bl = [&](int l, int salt) {
    return (l == 0 ? b0 : (l == 1 ? b1 : (l == 2 ? b2 : b3))) + opaque_zero(salt);
  };
  using Dm = BwdDims<HID, NL>;
  extern __shared__ float smem[];
  // LDS: per-layer padded accumulators (W then b), then the D / A staging.
  constexpr int kStageD = 64 * (16 > HID ? 16 : HID) + 0;
  int acc_off[NL], accb_off[NL];
  int tot = 0;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    acc_off[l] = tot;
    tot += Dm::out(l) * Dm::in(l);
    accb_off[l] = tot;
    tot += Dm::out(l);
  }
  float *acc = smem;
  float *Dst = smem + tot;        // [kBwdStage][dstride]
  constexpr int dstride = (HID > 16 ? HID : 16) + 4;
  float *Ast = Dst + kBwdStage * dstride;  // [kBwdStage][astride]
  constexpr int astride = (HID > 16 ? HID : 16) + 4;
  (void)kStageD;

  const int lane = threadIdx.x;
  for (int i = lane; i < tot; i += 64) acc[i] = 0.f;
  __syncthreads();

  const int n_out = a.dims[NL];
  const int n_levels = a.lat.n_levels;
  const int64_t n_chunks = (a.n + 63) / 64;
  for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
    const int salt = (int)chunk * 16;
    const int64_t s = chunk * 64 + lane;
    const bool valid = s < a.n;
    const float2 uv = a.uv[valid ? s : a.n - 1];

    // ---- forward: A[0] = x (padded to 16), A[l] = relu(z_{l-1})
    float x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = 0.f;
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) {
      if (k < n_levels) {
        const float3 c = sample_f32(a.lat.lv[k], uv.x, uv.y, a.lat.address);
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
    float h[NL - 1][HID];
    {
      const float *W = Wl(0, salt);
      const float *b = bl(0, salt);
      const int in0 = a.dims[0];
#pragma unroll
      for (int o = 0; o < HID; ++o) {
        float z = b[o];
#pragma unroll
        for (int k = 0; k < 14; ++k)
          if (k < in0) z = fmaf(W[o * in0 + k], x[k], z);
        h[0][o] = fmaxf(z, 0.f);
      }
    }
#pragma unroll
    for (int l = 1; l < NL - 1; ++l) {
      const float *W = Wl(l, salt + l);
      const float *b = bl(l, salt + l);
#pragma unroll
      for (int o = 0; o < HID; ++o) {
        float z = b[o];
#pragma unroll
        for (int k = 0; k < HID; ++k) z = fmaf(W[o * HID + k], h[l - 1][k], z);
        h[l][o] = fmaxf(z, 0.f);
      }
    }
    float d[HID > 16 ? HID : 16];
    {
      const float *W = Wl(NL - 1, salt + NL);
      const float *b = bl(NL - 1, salt + NL);
#pragma unroll
      for (int o = 0; o < 16; ++o) {
        d[o] = 0.f;
        if (o < n_out) {
          float z = b[o];
#pragma unroll
          for (int k = 0; k < HID; ++k) z = fmaf(W[o * HID + k], h[NL - 2][k], z);
          const float f = 1.0f / (1.0f + expf(-z));
          const float g = valid ? a.grad_out[s * n_out + o] : 0.f;
          d[o] = g * f * (1.0f - f);
        }
      }
    }

    // ---- backward through the layers
#pragma unroll
    for (int l = NL - 1; l >= 0; --l) {
      constexpr int dummy = 0;
      (void)dummy;
      const int M = Dm::out(l), K = Dm::in(l);
      // stage D_l and A_l of the chunk's samples, kBwdStage per round, and
      // accumulate their outer products
      for (int r = 0; r < 64 / kBwdStage; ++r) {
        if ((lane / kBwdStage) == r) {
          const int row = lane % kBwdStage;
#pragma unroll
          for (int o = 0; o < (l == NL - 1 ? 16 : HID); ++o) Dst[row * dstride + o] = d[o];
          if (l == 0) {
#pragma unroll
            for (int k = 0; k < 16; ++k) Ast[row * astride + k] = x[k];
          } else {
#pragma unroll
            for (int k = 0; k < HID; ++k) Ast[row * astride + k] = h[l - 1][k];
          }
        }
        __syncthreads();
        if (l == NL - 1) {
          accum_outer<16, HID>(Dst, dstride, Ast, astride, acc + acc_off[l], acc + accb_off[l], lane);
        } else if (l == 0) {
          accum_outer<HID, 16>(Dst, dstride, Ast, astride, acc + acc_off[l], acc + accb_off[l], lane);
        } else {
          accum_outer<HID, HID>(Dst, dstride, Ast, astride, acc + acc_off[l], acc + accb_off[l], lane);
        }
        __syncthreads();
      }
      (void)M;
      (void)K;
      if (l > 0) {
        // D_{l-1} = (W_l^T D_l) * [A_l > 0]
        const float *W = Wl(l, salt + 2 * NL + l);
        const int rows = (l == NL - 1) ? n_out : HID;
        float nd[HID];
#pragma unroll
        for (int k = 0; k < HID; ++k) nd[k] = 0.f;
#pragma unroll
        for (int o = 0; o < (l == NL - 1 ? 16 : HID); ++o) {
          if (o < rows) {
#pragma unroll
            for (int k = 0; k < HID; ++k) nd[k] = fmaf(W[o * HID + k], d[o], nd[k]);
          }
        }
#pragma unroll
        for (int k = 0; k < HID; ++k) d[k] = h[l - 1][k] > 0.f ? nd[k] : 0.f;
#pragma unroll
        for (int k = HID; k < (HID > 16 ? HID : 16); ++k) d[k] = 0.f;
      } else if (valid) {
        // dx = W_0^T D_0, spread onto the taps of every level
        const float *W = Wl(0, salt + 3 * NL);
        const int in0 = a.dims[0];
        float dx[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) dx[k] = 0.f;
#pragma unroll
        for (int o = 0; o < HID; ++o) {
#pragma unroll
          for (int k = 0; k < 12; ++k)
            if (k < in0 - 2) dx[k] = fmaf(W[o * in0 + k], d[o], dx[k]);
        }
#pragma unroll
        for (int k = 0; k < kMaxLevels; ++k) {
          if (k < n_levels) {
            const LevelArgs &L = a.lat.lv[k];
            const Taps t = tap_coords(uv.x, uv.y, L, a.lat.address);
            const float gx = 1.0f - t.fx, gy = 1.0f - t.fy;
            const float w[4] = {gx * gy, t.fx * gy, gx * t.fy, t.fx * t.fy};
            const int ii[4] = {t.i0, t.i1, t.i0, t.i1};
            const int jj[4] = {t.j0, t.j0, t.j1, t.j1};
            float *G = a.grad_lat[k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              float *p = G + ((int64_t)jj[q] * L.w + ii[q]) * 3;
              unsafeAtomicAdd(p + 0, w[q] * dx[3 * k + 0]);
              unsafeAtomicAdd(p + 1, w[q] * dx[3 * k + 1]);
              unsafeAtomicAdd(p + 2, w[q] * dx[3 * k + 2]);
            }
          }
        }
      }
    }
  }

  // ---- write this workgroup's partial sums (unpadded parameter order)
  __syncthreads();
  float *part = a.wpart + (int64_t)blockIdx.x * a.n_params;
  int poff = 0;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const int rows = a.dims[l + 1], cols = a.dims[l];
    const int K = Dm::in(l);
    for (int i = lane; i < rows * cols; i += 64) {
      const int r = i / cols, c = i % cols;
      part[poff + i] = acc[acc_off[l] + r * K + c];
    }
    poff += rows * cols;
    for (int i = lane; i < rows; i += 64) part[poff + i] = acc[accb_off[l] + i];
    poff += rows;
  }
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

template <int HID, int NL>
static size_t bwd_lds_bytes() {
  using Dm = BwdDims<HID, NL>;
  int tot = 0;
  for (int l = 0; l < NL; ++l) tot += Dm::out(l) * Dm::in(l) + Dm::out(l);
  const int stride = (HID > 16 ? HID : 16) + 4;
  return (size_t)(tot + 2 * kBwdStage * stride) * sizeof(float);
}

template <int HID, int NL>
static hipError_t launch_bwd(const BackwardArgs &a, hipStream_t st) {
  const size_t lds = bwd_lds_bytes<HID, NL>();
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL((backward_kernel<HID, NL>), dim3(a.n_blocks), dim3(64), lds, st, a, a.W[0], a.W[1], a.W[2],
                     a.W[3], a.b[0], a.b[1], a.b[2], a.b[3]);
  return hipGetLastError();
}

template <int HID>
static hipError_t launch_bwd_hid(const BackwardArgs &a, int nl, hipStream_t st) {
  switch (nl) {
    case 2: return launch_bwd<HID, 2>(a, st);
    case 3: return launch_bwd<HID, 3>(a, st);
    case 4: return launch_bwd<HID, 4>(a, st);
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
  switch (s.hid) {
    case 16: e = launch_bwd_hid<16>(a, s.n_layers, st); break;
    case 32: e = launch_bwd_hid<32>(a, s.n_layers, st); break;
    case 64: e = launch_bwd_hid<64>(a, s.n_layers, st); break;
    default: return hipErrorInvalidValue;
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
  return hipGetLastError();
}

int backward_n_params(const MlpShape &s) { return n_params_of(s); }

}  // namespace ntc
