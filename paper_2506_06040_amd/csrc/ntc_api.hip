// C ABI of libntc: argument validation, conversion to kernel arguments and
// launches. Every check runs on the host before anything is enqueued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ntc.h"
#include "ntc_internal.hpp"

using namespace ntc;

namespace {

thread_local char g_err[512];

ntc_status fail(ntc_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

ntc_status ok() {
  g_err[0] = 0;
  return NTC_OK;
}

ntc_status hip_fail(hipError_t e, const char *what) {
  return fail(NTC_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  static int cached[64] = {0};
  if (dev >= 0 && dev < 64 && cached[dev] > 0) return cached[dev];
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  if (dev >= 0 && dev < 64) cached[dev] = cus;
  return cus;
}

ntc_status check_latents(const ntc_latents *lat, bool need_bc1, bool need_f32) {
  if (!lat) return fail(NTC_E_NULL, "latents is NULL");
  if (lat->n_levels < 1 || lat->n_levels > NTC_MAX_LEVELS)
    return fail(NTC_E_SHAPE, "n_levels %d outside 1..%d", lat->n_levels, NTC_MAX_LEVELS);
  if (lat->format != NTC_LATENT_BC1 && lat->format != NTC_LATENT_F32)
    return fail(NTC_E_UNSUPPORTED, "latent format %d", lat->format);
  if (need_bc1 && lat->format != NTC_LATENT_BC1) return fail(NTC_E_UNSUPPORTED, "this call needs BC1 latents");
  if (need_f32 && lat->format != NTC_LATENT_F32) return fail(NTC_E_UNSUPPORTED, "this call needs float latents");
  if (lat->address != NTC_CLAMP && lat->address != NTC_WRAP)
    return fail(NTC_E_UNSUPPORTED, "address mode %d", lat->address);
  if (lat->reserved != 0) return fail(NTC_E_SHAPE, "reserved field must be 0");
  for (int k = 0; k < lat->n_levels; ++k) {
    const int w = lat->width[k], h = lat->height[k];
    if (w < 4 || h < 4 || w > 16384 || h > 16384)
      return fail(NTC_E_SHAPE, "level %d size %dx%d outside 4..16384", k, w, h);
    if (lat->format == NTC_LATENT_BC1 && ((w & 3) || (h & 3)))
      return fail(NTC_E_SHAPE, "BC1 level %d size %dx%d not a multiple of 4", k, w, h);
    if (!lat->data[k]) return fail(NTC_E_NULL, "latent level %d data is NULL", k);
    if (!aligned(lat->data[k], lat->format == NTC_LATENT_BC1 ? 8 : 4))
      return fail(NTC_E_ALIGN, "latent level %d data misaligned", k);
    for (int a = 0; a < 2; ++a) {
      const float s = lat->shift[k][a];
      if (!(s >= -1.0f && s <= 1.0f)) return fail(NTC_E_SHAPE, "level %d shift outside [-1, 1]", k);
    }
  }
  return NTC_OK;
}

ntc_status check_mlp_shape(const ntc_mlp *mlp, int n_levels, MlpShape *s) {
  if (!mlp) return fail(NTC_E_NULL, "mlp is NULL");
  const int L = mlp->n_layers;
  if (L < 2 || L > NTC_MAX_LAYERS) return fail(NTC_E_SHAPE, "n_layers %d outside 2..%d", L, NTC_MAX_LAYERS);
  if (n_levels > 0 && mlp->dims[0] != 3 * n_levels + 2)
    return fail(NTC_E_SHAPE, "dims[0] = %d but 3 * n_levels + 2 = %d", mlp->dims[0], 3 * n_levels + 2);
  if (mlp->dims[0] < 5 || mlp->dims[0] > 14 || (mlp->dims[0] - 2) % 3)
    return fail(NTC_E_SHAPE, "dims[0] = %d is not 3 * n_levels + 2 with 1 <= n_levels <= 4", mlp->dims[0]);
  const int hid = mlp->dims[1];
  if (hid != 16 && hid != 32 && hid != 64) return fail(NTC_E_UNSUPPORTED, "hidden width %d not in {16, 32, 64}", hid);
  for (int l = 1; l < L; ++l)
    if (mlp->dims[l] != hid) return fail(NTC_E_UNSUPPORTED, "hidden widths differ (dims[%d] = %d)", l, mlp->dims[l]);
  const int n_out = mlp->dims[L];
  if (n_out < 1 || n_out > 16) return fail(NTC_E_SHAPE, "output width %d outside 1..16", n_out);
  s->n_layers = L;
  s->in_dim = mlp->dims[0];
  s->hid = hid;
  s->n_out = n_out;
  return NTC_OK;
}

ntc_status check_mlp_weights(const ntc_mlp *mlp) {
  for (int l = 0; l < mlp->n_layers; ++l) {
    if (!mlp->W[l] || !mlp->b[l]) return fail(NTC_E_NULL, "layer %d weights or bias NULL", l);
    if (!aligned(mlp->W[l], 4) || !aligned(mlp->b[l], 4)) return fail(NTC_E_ALIGN, "layer %d misaligned", l);
  }
  return NTC_OK;
}

LatArgs to_lat_args(const ntc_latents *lat) {
  LatArgs a;
  memset(&a, 0, sizeof a);
  a.n_levels = lat->n_levels;
  a.format = lat->format;
  a.address = lat->address;
  for (int k = 0; k < NTC_MAX_LEVELS; ++k) {
    LevelArgs &L = a.lv[k];
    // Unused levels mirror level 0 so that every pointer stays valid, with
    // zero sampling scale and a shift of 1/2 (position 0): the matrix-core
    // decode samples all four levels without a branch, and such a level
    // always reads texels (0, 0) .. (1, 1) of level 0 into features whose
    // weights are zero.
    const bool used = k < lat->n_levels;
    const int src = used ? k : 0;
    L.w = lat->width[src];
    L.h = lat->height[src];
    L.bw = L.w / 4;
    L.fw = used ? (float)L.w : 0.0f;
    L.fh = used ? (float)L.h : 0.0f;
    L.sx = used ? lat->shift[src][0] : 0.5f;
    L.sy = used ? lat->shift[src][1] : 0.5f;
    if (lat->format == NTC_LATENT_BC1)
      L.bc1 = (const uint2 *)lat->data[src];
    else
      L.grid = (const float *)lat->data[src];
  }
  return a;
}

MlpPtrs to_mlp_ptrs(const ntc_mlp *mlp) {
  MlpPtrs p;
  memset(&p, 0, sizeof p);
  for (int l = 0; l < mlp->n_layers; ++l) {
    p.W[l] = mlp->W[l];
    p.b[l] = mlp->b[l];
  }
  for (int l = 0; l <= mlp->n_layers; ++l) p.dims[l] = mlp->dims[l];
  return p;
}

bool valid_compute(int c) { return c == NTC_F32 || c == NTC_F16 || c == NTC_BF16 || c == NTC_FP8_E4M3; }

}  // namespace

extern "C" {

const char *ntc_status_string(ntc_status s) {
  switch (s) {
    case NTC_OK: return "NTC_OK";
    case NTC_E_NULL: return "NTC_E_NULL: required pointer is NULL";
    case NTC_E_SHAPE: return "NTC_E_SHAPE: inconsistent or out-of-range sizes";
    case NTC_E_UNSUPPORTED: return "NTC_E_UNSUPPORTED: not implemented for these arguments";
    case NTC_E_WORKSPACE: return "NTC_E_WORKSPACE: buffer too small";
    case NTC_E_HIP: return "NTC_E_HIP: HIP runtime or launch failure";
    case NTC_E_ALIGN: return "NTC_E_ALIGN: misaligned device pointer";
  }
  return "unknown ntc_status";
}

const char *ntc_last_error(void) { return g_err; }

int32_t ntc_version(void) { return 10000 * 0 + 100 * 4 + 0; }

ntc_status ntc_mlp_pack_size(const ntc_mlp *mlp, int32_t compute, size_t *bytes) {
  if (!bytes) return fail(NTC_E_NULL, "bytes is NULL");
  if (!valid_compute(compute)) return fail(NTC_E_UNSUPPORTED, "compute type %d", compute);
  MlpShape s;
  ntc_status st = check_mlp_shape(mlp, 0, &s);
  if (st) return st;
  *bytes = pack_layout(s, compute).total;
  return ok();
}

ntc_status ntc_mlp_pack(const ntc_mlp *mlp, int32_t compute, const float *act_amax, void *packed, size_t bytes,
                        void *stream) {
  if (!valid_compute(compute)) return fail(NTC_E_UNSUPPORTED, "compute type %d", compute);
  MlpShape s;
  ntc_status st = check_mlp_shape(mlp, 0, &s);
  if (st) return st;
  if ((st = check_mlp_weights(mlp))) return st;
  if (!packed) return fail(NTC_E_NULL, "packed is NULL");
  if (!aligned(packed, 256)) return fail(NTC_E_ALIGN, "packed must be 256-byte aligned");
  const PackLayout lay = pack_layout(s, compute);
  if (bytes < lay.total) return fail(NTC_E_WORKSPACE, "packed needs %zu bytes, got %zu", lay.total, bytes);
  if (compute == NTC_FP8_E4M3) {
    if (!act_amax) return fail(NTC_E_NULL, "FP8 packing needs act_amax");
    if (!aligned(act_amax, 4)) return fail(NTC_E_ALIGN, "act_amax misaligned");
  }
  hipError_t e = launch_pack(s, to_mlp_ptrs(mlp), compute, act_amax, (uint8_t *)packed, lay, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pack launch");
  return ok();
}

ntc_status ntc_calibrate_fp8(const ntc_latents *lat, const ntc_mlp *mlp, const void *packed_f32,
                             const float *uv, int64_t n, float *act_amax, void *stream) {
  ntc_status st = check_latents(lat, false, false);
  if (st) return st;
  MlpShape s;
  if ((st = check_mlp_shape(mlp, lat->n_levels, &s))) return st;
  if (!packed_f32 || !uv || !act_amax) return fail(NTC_E_NULL, "packed_f32, uv or act_amax is NULL");
  if (!aligned(packed_f32, 256)) return fail(NTC_E_ALIGN, "packed_f32 must be 256-byte aligned");
  if (!aligned(uv, 8) || !aligned(act_amax, 4)) return fail(NTC_E_ALIGN, "uv or act_amax misaligned");
  if (n < 1) return fail(NTC_E_SHAPE, "calibration needs n >= 1");
  DecodeArgs a;
  memset(&a, 0, sizeof a);
  a.lat = to_lat_args(lat);
  a.packed = (const uint8_t *)packed_f32;
  a.uv = (const float2 *)uv;
  a.n = n;
  a.n_tiles = (n + 63) / 64;
  a.n_out = s.n_out;
  a.n_layers = s.n_layers;
  a.lay = pack_layout(s, NTC_F32);
  hipError_t e = launch_fill_f32(act_amax, s.n_layers, 0.0f, (hipStream_t)stream);
  if (e == hipSuccess) e = launch_decode_plain(a, s, act_amax, device_cus(), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "calibration launch");
  return ok();
}

ntc_status ntc_decode(const ntc_latents *lat, const ntc_mlp *mlp, int32_t compute, const void *packed,
                      const float *uv, int64_t n, void *out, int32_t out_dtype, const ntc_tile_cfg *cfg,
                      void *stream) {
  if (!valid_compute(compute)) return fail(NTC_E_UNSUPPORTED, "compute type %d", compute);
  ntc_status st = check_latents(lat, compute != NTC_F32, false);
  if (st) return st;
  MlpShape s;
  if ((st = check_mlp_shape(mlp, lat->n_levels, &s))) return st;
  if (out_dtype != NTC_F32 && out_dtype != NTC_F16) return fail(NTC_E_UNSUPPORTED, "out dtype %d", out_dtype);
  if (n < 0) return fail(NTC_E_SHAPE, "n < 0");
  if (n > ((int64_t)1 << 40)) return fail(NTC_E_SHAPE, "n too large");
  if (!packed || !uv || !out) {
    if (n == 0) return ok();
    return fail(NTC_E_NULL, "packed, uv or out is NULL");
  }
  if (!aligned(packed, 256)) return fail(NTC_E_ALIGN, "packed must be 256-byte aligned");
  if (!aligned(uv, 8)) return fail(NTC_E_ALIGN, "uv must be 8-byte aligned");
  if (!aligned(out, 16)) return fail(NTC_E_ALIGN, "out must be 16-byte aligned");
  const int span = decode_span_tiles(s.hid, s.n_layers, compute);
  int stage_cap = 1024, waves_per_cu = 8, tiles_per_iter = span;
  if (cfg) {
    if (cfg->waves_per_cu) waves_per_cu = cfg->waves_per_cu;
    if (cfg->stage_capacity) stage_cap = cfg->stage_capacity;
    if (cfg->tiles_per_iter) tiles_per_iter = cfg->tiles_per_iter;
    if (tiles_per_iter != span)
      return fail(NTC_E_UNSUPPORTED, "tiles_per_iter %d (compiled for %d for this network shape)", tiles_per_iter,
                  span);
  }
  if (waves_per_cu < 1 || waves_per_cu > 1024)
    return fail(NTC_E_SHAPE, "waves_per_cu %d outside 1..1024", waves_per_cu);
  if (stage_cap < 64 || stage_cap > 4096) return fail(NTC_E_SHAPE, "stage_capacity %d outside 64..4096", stage_cap);
  if (n == 0) return ok();

  DecodeArgs a;
  memset(&a, 0, sizeof a);
  a.lat = to_lat_args(lat);
  a.packed = (const uint8_t *)packed;
  a.uv = (const float2 *)uv;
  a.out = out;
  a.n = n;
  a.n_tiles = (n + 63) / 64;
  a.n_out = s.n_out;
  a.out_f16 = out_dtype == NTC_F16;
  a.stage_cap = stage_cap;
  a.n_layers = s.n_layers;
  a.lay = pack_layout(s, compute);
  const int cus = device_cus();
  hipError_t e;
  if (compute == NTC_F32 && lat->format == NTC_LATENT_F32 && s.n_layers <= 4)
    e = launch_forward_f32(a, s, (hipStream_t)stream);
  else if (compute == NTC_F32)
    e = launch_decode_plain(a, s, nullptr, cus, (hipStream_t)stream);
  else
    e = launch_decode_mfma(a, s, compute, cus * waves_per_cu, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "decode launch");
  return ok();
}

ntc_status ntc_bc1_decode_texels(const ntc_latents *lat, int32_t level, float *out, uint16_t *numer,
                                 void *stream) {
  ntc_status st = check_latents(lat, true, false);
  if (st) return st;
  if (level < 0 || level >= lat->n_levels) return fail(NTC_E_SHAPE, "level %d outside 0..%d", level, lat->n_levels - 1);
  if (!out && !numer) return fail(NTC_E_NULL, "out and numer are both NULL");
  if ((out && !aligned(out, 4)) || (numer && !aligned(numer, 2))) return fail(NTC_E_ALIGN, "output misaligned");
  const LatArgs a = to_lat_args(lat);
  hipError_t e = launch_bc1_texels(a.lv[level], out, numer, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "texel launch");
  return ok();
}

ntc_status ntc_decode_filtered(const ntc_latent_mips *lat, const ntc_mlp *mlp, const void *packed, const float *uv,
                               const float *duv, int64_t n, void *out, int32_t out_dtype, int32_t filter,
                               int32_t max_aniso, void *stream) {
  if (!lat) return fail(NTC_E_NULL, "latents is NULL");
  if (lat->n_levels < 1 || lat->n_levels > NTC_MAX_LEVELS)
    return fail(NTC_E_SHAPE, "n_levels %d outside 1..%d", lat->n_levels, NTC_MAX_LEVELS);
  MlpShape s;
  ntc_status st = check_mlp_shape(mlp, lat->n_levels, &s);
  if (st) return st;
  if (s.n_layers > 4) return fail(NTC_E_UNSUPPORTED, "filtered decode supports at most 4 layers");
  if (filter != NTC_FILTER_TRILINEAR && filter != NTC_FILTER_ANISOTROPIC)
    return fail(NTC_E_UNSUPPORTED, "filter %d", filter);
  if (max_aniso < 1 || max_aniso > NTC_MAX_ANISO) return fail(NTC_E_SHAPE, "max_aniso %d outside 1..%d", max_aniso, NTC_MAX_ANISO);
  if (out_dtype != NTC_F32 && out_dtype != NTC_F16) return fail(NTC_E_UNSUPPORTED, "out dtype %d", out_dtype);
  if (n < 0 || n > ((int64_t)1 << 40)) return fail(NTC_E_SHAPE, "n %lld outside 0..2^40", (long long)n);
  for (int k = 0; k < lat->n_levels; ++k) {
    const int w = lat->width[k], h = lat->height[k], nm = lat->n_mips[k];
    if (nm < 1 || nm > NTC_MAX_MIPS) return fail(NTC_E_SHAPE, "level %d: n_mips %d outside 1..%d", k, nm, NTC_MAX_MIPS);
    if (w < 4 || h < 4 || w > 65536 || h > 65536)
      return fail(NTC_E_SHAPE, "level %d: %d x %d outside 4..65536", k, w, h);
    for (int m = 0; m < nm; ++m) {
      if (((w >> m) & 3) || ((h >> m) & 3) || (w >> m) < 4 || (h >> m) < 4 || ((w >> m) << m) != w ||
          ((h >> m) << m) != h)
        return fail(NTC_E_SHAPE, "level %d mip %d: %d x %d is not a multiple of 4 of at least 4", k, m, w >> m,
                    h >> m);
      if (!lat->data[k][m]) return fail(NTC_E_NULL, "level %d mip %d has no data", k, m);
      if (!aligned(lat->data[k][m], 8)) return fail(NTC_E_ALIGN, "level %d mip %d misaligned", k, m);
    }
    if (!(fabsf(lat->shift[k][0]) <= 1.0f) || !(fabsf(lat->shift[k][1]) <= 1.0f))
      return fail(NTC_E_SHAPE, "level %d: |shift| > 1", k);
  }
  if (n == 0) return ok();
  if (!packed || !uv || !duv || !out) return fail(NTC_E_NULL, "packed, uv, duv or out is NULL");
  if (!aligned(packed, 256) || !aligned(uv, 8) || !aligned(duv, 16) || !aligned(out, 16))
    return fail(NTC_E_ALIGN, "misaligned packed, uv, duv or out");
  FilterArgs f;
  memset(&f, 0, sizeof f);
  DecodeArgs &a = f.d;
  a.packed = (const uint8_t *)packed;
  a.uv = (const float2 *)uv;
  a.out = out;
  a.n = n;
  a.n_tiles = (n + 63) / 64;
  a.n_out = s.n_out;
  a.out_f16 = out_dtype == NTC_F16;
  a.n_layers = s.n_layers;
  a.lay = pack_layout(s, NTC_F16);
  f.duv = (const float4 *)duv;
  f.n_levels = lat->n_levels;
  f.filter = filter;
  f.max_aniso = max_aniso;
  for (int k = 0; k < NTC_MAX_LEVELS; ++k) {
    // unused levels and mips mirror valid ones so that every pointer stays valid
    const int src = k < lat->n_levels ? k : 0;
    f.n_mips[k] = lat->n_mips[src];
    f.w0[k] = (float)lat->width[src];
    f.h0[k] = (float)lat->height[src];
    f.sx[k] = lat->shift[src][0];
    f.sy[k] = lat->shift[src][1];
    for (int m = 0; m < kMaxMips; ++m) {
      const int ms = m < lat->n_mips[src] ? m : lat->n_mips[src] - 1;
      MipArgs &M = f.mip[k][m];
      M.bc1 = (const uint2 *)lat->data[src][ms];
      M.w = lat->width[src] >> ms;
      M.h = lat->height[src] >> ms;
      M.bw = M.w / 4;
      M.fw = (float)M.w;
      M.fh = (float)M.h;
    }
  }
  // one level-of-detail computation per pixel when every level is level 0
  // scaled by a power of two on both axes
  f.shared_lod = 1;
  for (int k = 0; k < lat->n_levels; ++k) {
    int e = 0;
    const int w = lat->width[k], h = lat->height[k], w0 = lat->width[0], h0 = lat->height[0];
    if (w <= w0) {
      while ((w << e) < w0) ++e;
      if ((w << e) != w0 || (h << e) != h0) f.shared_lod = 0;
      f.lod_shift[k] = (float)e;
      f.shift_i[k] = e;
    } else {
      while ((w0 << e) < w) ++e;
      if ((w0 << e) != w || (h0 << e) != h) f.shared_lod = 0;
      f.lod_shift[k] = -(float)e;
      f.shift_i[k] = -e;
    }
  }
  hipError_t e = launch_decode_filtered(f, s, device_cus() * 8, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "filtered decode launch");
  return ok();
}

static ntc_status check_qat_level(const float *params, int32_t width, int32_t height) {
  if (!params) return fail(NTC_E_NULL, "params is NULL");
  if (!aligned(params, 4)) return fail(NTC_E_ALIGN, "params misaligned");
  if (width < 4 || height < 4 || (width & 3) || (height & 3) || width > 16384 || height > 16384)
    return fail(NTC_E_SHAPE, "level %d x %d: sides must be multiples of 4 in 4..16384", width, height);
  return NTC_OK;
}

ntc_status ntc_qat_texels(const float *params, int32_t width, int32_t height, float *texels, void *stream) {
  ntc_status st = check_qat_level(params, width, height);
  if (st) return st;
  if (!texels) return fail(NTC_E_NULL, "texels is NULL");
  if (!aligned(texels, 4)) return fail(NTC_E_ALIGN, "texels misaligned");
  hipError_t e = launch_qat_texels(params, width, height, texels, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "qat texels launch");
  return ok();
}

ntc_status ntc_qat_backward(const float *params, int32_t width, int32_t height, const float *grad_texels,
                            float *grad_params, void *stream) {
  ntc_status st = check_qat_level(params, width, height);
  if (st) return st;
  if (!grad_texels || !grad_params) return fail(NTC_E_NULL, "grad_texels or grad_params is NULL");
  if (!aligned(grad_texels, 4) || !aligned(grad_params, 4)) return fail(NTC_E_ALIGN, "gradients misaligned");
  hipError_t e = launch_qat_backward(params, width, height, grad_texels, grad_params, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "qat backward launch");
  return ok();
}

ntc_status ntc_qat_export_bc1(const float *params, int32_t width, int32_t height, uint64_t *blocks, void *stream) {
  ntc_status st = check_qat_level(params, width, height);
  if (st) return st;
  if (!blocks) return fail(NTC_E_NULL, "blocks is NULL");
  if (!aligned(blocks, 8)) return fail(NTC_E_ALIGN, "blocks must be 8-byte aligned");
  hipError_t e = launch_qat_export(params, width, height, blocks, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "qat export launch");
  return ok();
}

static ntc_status check_frame(int32_t width, int32_t height, int32_t n_mats) {
  if (width < 1 || height < 1 || width > 32768 || height > 32768 || (int64_t)width * height >= ((int64_t)1 << 31))
    return fail(NTC_E_SHAPE, "frame %d x %d outside 1..32768 per side or 2^31 pixels", width, height);
  if (n_mats < 1 || n_mats > NTC_MAX_CLASSIFY_MATERIALS)
    return fail(NTC_E_SHAPE, "n_mats %d outside 1..%d", n_mats, NTC_MAX_CLASSIFY_MATERIALS);
  return NTC_OK;
}

ntc_status ntc_classify_workspace(int32_t width, int32_t height, int32_t n_mats, size_t *bytes) {
  if (!bytes) return fail(NTC_E_NULL, "bytes is NULL");
  ntc_status st = check_frame(width, height, n_mats);
  if (st) return st;
  *bytes = classify_workspace_bytes(width, height, n_mats);
  return ok();
}

ntc_status ntc_classify(const uint16_t *mat_ids, int32_t width, int32_t height, int32_t n_mats, int32_t *pixel_list,
                        int32_t *mat_offsets, int32_t *mat_simple, uint8_t *tile_class, void *workspace,
                        size_t ws_bytes, void *stream) {
  ntc_status st = check_frame(width, height, n_mats);
  if (st) return st;
  if (!mat_ids || !pixel_list || !mat_offsets || !mat_simple || !workspace)
    return fail(NTC_E_NULL, "mat_ids, pixel_list, mat_offsets, mat_simple or workspace is NULL");
  if (!aligned(mat_ids, 2) || !aligned(pixel_list, 4) || !aligned(mat_offsets, 4) || !aligned(mat_simple, 4) ||
      !aligned(workspace, 256))
    return fail(NTC_E_ALIGN, "misaligned classification buffer");
  const size_t need = classify_workspace_bytes(width, height, n_mats);
  if (ws_bytes < need) return fail(NTC_E_WORKSPACE, "classification needs %zu workspace bytes, got %zu", need, ws_bytes);
  hipError_t e = launch_classify(mat_ids, width, height, n_mats, pixel_list, mat_offsets, mat_simple, tile_class,
                                 workspace, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "classification launch");
  return ok();
}

ntc_status ntc_classify_noalloc(const uint16_t *mat_ids, int32_t width, int32_t height, int32_t n_mats,
                                int32_t *pixel_list, int32_t *mat_offsets, int32_t *mat_simple, uint8_t *tile_class,
                                void *stream) {
  ntc_status st = check_frame(width, height, n_mats);
  if (st) return st;
  if (!mat_ids || !pixel_list || !mat_offsets || !mat_simple)
    return fail(NTC_E_NULL, "mat_ids, pixel_list, mat_offsets or mat_simple is NULL");
  if (!aligned(mat_ids, 2) || !aligned(pixel_list, 4) || !aligned(mat_offsets, 4) || !aligned(mat_simple, 4))
    return fail(NTC_E_ALIGN, "misaligned classification buffer");
  const size_t need = classify_workspace_bytes(width, height, n_mats);
  if (need > classify_scratch_bytes())
    return fail(NTC_E_WORKSPACE,
                "classification of %d x %d pixels with %d materials needs %zu bytes of scratch; "
                "ntc_classify_noalloc holds %zu (use ntc_classify with a workspace)",
                width, height, n_mats, need, classify_scratch_bytes());
  void *ws = nullptr;
  hipError_t e = classify_scratch(&ws);
  if (e != hipSuccess) return hip_fail(e, "scratch address");
  e = launch_classify(mat_ids, width, height, n_mats, pixel_list, mat_offsets, mat_simple, tile_class, ws,
                      (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "classification launch");
  return ok();
}

ntc_status ntc_gather_uv(const float *uv_image, const int32_t *pixel_list, int64_t n, float *uv, void *stream) {
  if (n < 0) return fail(NTC_E_SHAPE, "n < 0");
  if (n == 0) return ok();
  if (!uv_image || !pixel_list || !uv) return fail(NTC_E_NULL, "uv_image, pixel_list or uv is NULL");
  if (!aligned(uv_image, 8) || !aligned(uv, 8) || !aligned(pixel_list, 4)) return fail(NTC_E_ALIGN, "misaligned");
  hipError_t e = launch_gather_uv(uv_image, pixel_list, n, uv, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gather launch");
  return ok();
}

ntc_status ntc_scatter_rows(const void *rows, const int32_t *pixel_list, int64_t n, int32_t channels, int32_t dtype,
                            void *image, void *stream) {
  if (n < 0) return fail(NTC_E_SHAPE, "n < 0");
  if (channels < 1 || channels > 16) return fail(NTC_E_SHAPE, "channels %d outside 1..16", channels);
  if (dtype != NTC_F32 && dtype != NTC_F16) return fail(NTC_E_UNSUPPORTED, "dtype %d", dtype);
  if (n == 0) return ok();
  if (!rows || !pixel_list || !image) return fail(NTC_E_NULL, "rows, pixel_list or image is NULL");
  const int eb = dtype == NTC_F32 ? 4 : 2;
  if (!aligned(rows, eb) || !aligned(image, eb) || !aligned(pixel_list, 4)) return fail(NTC_E_ALIGN, "misaligned");
  hipError_t e = launch_scatter_rows(rows, pixel_list, n, channels, eb, image, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "scatter launch");
  return ok();
}

ntc_status ntc_decode_backward_workspace(const ntc_latents *lat, const ntc_mlp *mlp, int64_t n, size_t *bytes) {
  if (!bytes) return fail(NTC_E_NULL, "bytes is NULL");
  ntc_status st = check_latents(lat, false, true);
  if (st) return st;
  MlpShape s;
  if ((st = check_mlp_shape(mlp, lat->n_levels, &s))) return st;
  if (s.n_layers > 4) return fail(NTC_E_UNSUPPORTED, "backward supports at most 4 layers");
  if (n < 0 || n > ((int64_t)1 << 36)) return fail(NTC_E_SHAPE, "n = %lld out of range", (long long)n);
  *bytes = backward_layout(s, to_lat_args(lat), n).total;
  return ok();
}

ntc_status ntc_decode_backward(const ntc_latents *lat, const ntc_mlp *mlp, const float *uv, int64_t n,
                               const float *grad_out, float *const *grad_W, float *const *grad_b,
                               float *const *grad_latents, void *workspace, size_t ws_bytes, void *stream) {
  ntc_status st = check_latents(lat, false, true);
  if (st) return st;
  MlpShape s;
  if ((st = check_mlp_shape(mlp, lat->n_levels, &s))) return st;
  if ((st = check_mlp_weights(mlp))) return st;
  if (s.n_layers > 4) return fail(NTC_E_UNSUPPORTED, "backward supports at most 4 layers");
  if (n < 0 || n > ((int64_t)1 << 36)) return fail(NTC_E_SHAPE, "n = %lld out of range", (long long)n);
  if (!grad_W || !grad_b || !grad_latents) return fail(NTC_E_NULL, "gradient pointer arrays are NULL");
  for (int l = 0; l < s.n_layers; ++l) {
    if (!grad_W[l] || !grad_b[l]) return fail(NTC_E_NULL, "gradient of layer %d is NULL", l);
    if (!aligned(grad_W[l], 4) || !aligned(grad_b[l], 4)) return fail(NTC_E_ALIGN, "gradient of layer %d misaligned", l);
  }
  for (int k = 0; k < lat->n_levels; ++k) {
    if (!grad_latents[k]) return fail(NTC_E_NULL, "latent gradient %d is NULL", k);
    if (!aligned(grad_latents[k], 4)) return fail(NTC_E_ALIGN, "latent gradient %d misaligned", k);
  }
  const LatArgs la = to_lat_args(lat);
  const BwdLayout lay = backward_layout(s, la, n);
  const size_t need = lay.total;
  if (!workspace) return fail(NTC_E_NULL, "workspace is NULL");
  if (ws_bytes < need) return fail(NTC_E_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
  if (!aligned(workspace, 256)) return fail(NTC_E_ALIGN, "workspace must be 256-byte aligned");
  if (n > 0) {
    if (!uv || !grad_out) return fail(NTC_E_NULL, "uv or grad_out is NULL");
    if (!aligned(uv, 8) || !aligned(grad_out, 4)) return fail(NTC_E_ALIGN, "uv or grad_out misaligned");
  }
  hipStream_t hs = (hipStream_t)stream;
  if (n == 0) {
    // no samples: every gradient is zero
    hipError_t e = hipSuccess;
    for (int l = 0; l < s.n_layers && e == hipSuccess; ++l) {
      e = launch_fill_f32(grad_W[l], (int64_t)mlp->dims[l] * mlp->dims[l + 1], 0.0f, hs);
      if (e == hipSuccess) e = launch_fill_f32(grad_b[l], mlp->dims[l + 1], 0.0f, hs);
    }
    for (int k = 0; k < lat->n_levels && e == hipSuccess; ++k)
      e = launch_fill_f32(grad_latents[k], (int64_t)lat->width[k] * lat->height[k] * 3, 0.0f, hs);
    if (e != hipSuccess) return hip_fail(e, "backward fill");
    return ok();
  }
  BackwardArgs a;
  memset(&a, 0, sizeof a);
  a.lat = la;
  for (int l = 0; l < s.n_layers; ++l) {
    a.W[l] = mlp->W[l];
    a.b[l] = mlp->b[l];
  }
  for (int l = 0; l <= s.n_layers; ++l) a.dims[l] = mlp->dims[l];
  a.n_layers = s.n_layers;
  a.uv = (const float2 *)uv;
  a.grad_out = grad_out;
  for (int k = 0; k < lat->n_levels; ++k) a.grad_lat[k] = grad_latents[k];
  uint8_t *ws = (uint8_t *)workspace;
  a.wpart = (float *)(ws + lay.wpart_off);
  a.dx = (float *)(ws + lay.dx_off);
  a.bin_count = (int32_t *)(ws + lay.count_off);
  a.bin_cursor = (int32_t *)(ws + lay.cursor_off);
  a.perm = (int32_t *)(ws + lay.perm_off);
  a.n = n;
  a.n_params = lay.n_params;
  a.n_blocks = lay.n_blocks;
  a.n_feat = lay.n_feat;
  a.bin_tex = lay.bin_tex;
  a.bins_x = lay.bins_x;
  a.bins_y = lay.bins_y;
  a.n_bins = lay.n_bins;
  a.bin_lds = lay.bin_lds;
  hipError_t e = launch_backward(a, s, grad_W, grad_b, hs);
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return ok();
}

namespace {

struct BatchSetup {
  std::vector<BatchMaterial> mats;
  int item_tiles = 64;
  int n_waves = 1;
  int stage_cap = 1024;
  int64_t n_items = 0;
};

ntc_status setup_batch(const ntc_material *mats, int32_t n_mats, const ntc_batch_cfg *cfg, BatchSetup *b) {
  if (!mats) return fail(NTC_E_NULL, "materials is NULL");
  if (n_mats < 1 || n_mats > 65536) return fail(NTC_E_SHAPE, "n_mats %d outside 1..65536", n_mats);
  int item_px = 4096, wpc = 8, cap = 1024, cus = 256;
  if (cfg) {
    if (cfg->item_pixels) item_px = cfg->item_pixels;
    if (cfg->waves_per_cu) wpc = cfg->waves_per_cu;
    if (cfg->stage_capacity) cap = cfg->stage_capacity;
    if (cfg->n_cus) cus = cfg->n_cus;
  }
  if (item_px < 64 || item_px > 65536 || (item_px & 63)) return fail(NTC_E_SHAPE, "item_pixels %d", item_px);
  if (wpc < 1 || wpc > 1024) return fail(NTC_E_SHAPE, "waves_per_cu %d outside 1..1024", wpc);
  if (cap < 64 || cap > 4096) return fail(NTC_E_SHAPE, "stage_capacity %d outside 64..4096", cap);
  if (cus < 1 || cus > 4096) return fail(NTC_E_SHAPE, "n_cus %d", cus);
  b->mats.resize(n_mats);
  std::vector<int64_t> npx(n_mats);
  for (int m = 0; m < n_mats; ++m) {
    const ntc_material &M = mats[m];
    ntc_status st = check_latents(&M.lat, true, false);
    if (st) return fail(st, "material %d: %s", m, g_err);
    MlpShape s;
    if ((st = check_mlp_shape(&M.mlp, M.lat.n_levels, &s))) return fail(st, "material %d: %s", m, g_err);
    const int sid = shape_id_of(s.hid, s.n_layers);
    if (sid < 0) return fail(NTC_E_UNSUPPORTED, "material %d: batched decode supports 2..4 layers", m);
    if (M.n < 1 || M.n > ((int64_t)1 << 40)) return fail(NTC_E_SHAPE, "material %d: n = %lld", m, (long long)M.n);
    if (!M.packed || !M.uv || !M.out) return fail(NTC_E_NULL, "material %d: packed, uv or out is NULL", m);
    if (!aligned(M.packed, 256) || !aligned(M.uv, 8) || !aligned(M.out, 16))
      return fail(NTC_E_ALIGN, "material %d: misaligned pointer", m);
    if (M.out_dtype != NTC_F32 && M.out_dtype != NTC_F16)
      return fail(NTC_E_UNSUPPORTED, "material %d: out dtype %d", m, M.out_dtype);
    if (M.pixel_index) {
      const int64_t esz = M.out_dtype == NTC_F16 ? 2 : 4;
      if (!aligned(M.pixel_index, 4)) return fail(NTC_E_ALIGN, "material %d: pixel_index misaligned", m);
      if (M.image_pixels < 1 || M.image_pixels * s.n_out * esz >= ((int64_t)1 << 30) ||
          M.image_pixels * 8 >= ((int64_t)1 << 30))
        return fail(NTC_E_SHAPE, "material %d: image_pixels %lld outside 1..2^30 bytes of uv and output", m,
                    (long long)M.image_pixels);
      if (M.n > ((int64_t)1 << 28)) return fail(NTC_E_SHAPE, "material %d: indexed n above 2^28", m);
    }
    BatchMaterial &B = b->mats[m];
    memset(&B, 0, sizeof B);
    B.a.lat = to_lat_args(&M.lat);
    B.a.packed = (const uint8_t *)M.packed;
    B.a.uv = (const float2 *)M.uv;
    B.a.out = M.out;
    B.a.n = M.n;
    B.a.n_tiles = (M.n + 63) / 64;
    B.a.n_out = s.n_out;
    B.a.out_f16 = M.out_dtype == NTC_F16;
    B.a.stage_cap = cap;
    B.a.n_layers = s.n_layers;
    B.a.lay = pack_layout(s, NTC_F16);
    B.a.pix = M.pixel_index;
    B.a.img_px = M.pixel_index ? M.image_pixels : 0;
    B.shape_id = sid;
    B.hid = s.hid;
    B.n_layers = s.n_layers;
    npx[m] = M.n;
  }
  b->item_tiles = item_px / 64;
  b->n_items = count_items(npx.data(), n_mats, b->item_tiles);
  if (b->n_items > (int64_t)1 << 30) return fail(NTC_E_SHAPE, "too many work items");
  b->n_waves = plan_waves(b->n_items, cus, wpc);
  b->stage_cap = cap;
  return NTC_OK;
}

}  // namespace

ntc_status ntc_batched_plan_size(const ntc_material *mats, int32_t n_mats, const ntc_batch_cfg *cfg, size_t *bytes) {
  if (!bytes) return fail(NTC_E_NULL, "bytes is NULL");
  BatchSetup b;
  ntc_status st = setup_batch(mats, n_mats, cfg, &b);
  if (st) return st;
  *bytes = plan_bytes(n_mats, b.n_items, b.n_waves);
  return ok();
}

ntc_status ntc_batched_plan(const ntc_material *mats, int32_t n_mats, const ntc_batch_cfg *cfg, void *plan_host,
                            size_t bytes) {
  BatchSetup b;
  ntc_status st = setup_batch(mats, n_mats, cfg, &b);
  if (st) return st;
  if (!plan_host) return fail(NTC_E_NULL, "plan_host is NULL");
  const size_t need = plan_bytes(n_mats, b.n_items, b.n_waves);
  if (bytes < need) return fail(NTC_E_WORKSPACE, "plan needs %zu bytes, got %zu", need, bytes);
  build_plan(b.mats.data(), n_mats, b.item_tiles, b.n_waves, b.stage_cap, (uint8_t *)plan_host, need);
  return ok();
}

ntc_status ntc_decode_batched(const void *plan_host, const void *plan_dev, size_t bytes, void *stream) {
  if (!plan_host || !plan_dev) return fail(NTC_E_NULL, "plan_host or plan_dev is NULL");
  if (bytes < sizeof(BatchPlanHeader)) return fail(NTC_E_WORKSPACE, "plan too small");
  if (!aligned(plan_dev, 256)) return fail(NTC_E_ALIGN, "plan_dev must be 256-byte aligned");
  BatchPlanHeader h;
  memcpy(&h, plan_host, sizeof h);
  if (h.magic != kPlanMagic || h.version != kPlanVersion) return fail(NTC_E_SHAPE, "not a plan image");
  if (h.total_bytes > bytes) return fail(NTC_E_WORKSPACE, "plan image truncated");
  if (h.n_waves < 1 || h.stage_cap < 64 || h.stage_cap > 4096) return fail(NTC_E_SHAPE, "corrupt plan header");
  hipError_t e = launch_decode_batched((const uint8_t *)plan_dev, h, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "batched launch");
  return ok();
}

}  // extern "C"
