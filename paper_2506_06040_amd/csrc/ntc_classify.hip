// Tile classification of a frame and per-MLP pixel lists (Sec. 4, "Tile-based
// classification", Algorithm 1).
//
// The paper classifies the 8x4 pixel tiles of the screen by the material ids
// of their pixels: no neural pixel, a single network with more than 16
// pixels ("simple", decoded as a tile), or anything else ("mixed", whose
// pixels are regrouped by network into dense tiles); it appends tiles and
// pixels to lists with global atomics, and notes that these do not scale
// when many tiles are mixed. Here the lists are built without global
// atomics and in a fixed order, so that the result is deterministic:
//   1. count: one wavefront per chunk of 128 consecutive tiles (two tiles per
//      step, lane = pixel) classifies each tile and counts its valid pixels
//      per key (material, kind), kind 0 = simple tile, 1 = other;
//   2. scan: per key, exclusive prefix over chunks; then over materials;
//   3. write: the same walk ranks each pixel inside its key group (ballot and
//      lane-count) and writes its index.
// Output: the valid pixels grouped by material; inside a material, first
// the pixels of its simple tiles, then its other pixels, each part in tile
// order and row-major inside a tile.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ntc_internal.hpp"

namespace ntc {

// Scratch of the allocation-free entry point (ntc_classify_noalloc): the
// per-chunk key counts and the key totals of one classification, in a
// file-scope device array of which every GPU holds its own copy for the
// life of the process. Every entry the passes read is written earlier in
// the same call, so nothing needs clearing between calls.
constexpr size_t kClassifyScratchBytes = size_t(8) << 20;
static __device__ __align__(256) int32_t scratch[kClassifyScratchBytes / sizeof(int32_t)];

namespace {

constexpr int kTilesPerChunk = 128;  // two tiles per wavefront step, 64 steps
constexpr int kScanThreads = 256;

struct ClassifyArgs {
  const uint16_t *mat;   // [h][w]
  int32_t w, h, tw, n_tiles, n_chunks, n_mats;
  int32_t *counts;       // [2 n_mats][n_chunks]: count, then exclusive offset
  int32_t *totals;       // [2 n_mats]
  int32_t *mat_offsets;  // [n_mats + 1]
  int32_t *mat_simple;   // [n_mats]
  int32_t *list;         // [valid pixels]
  uint8_t *tile_class;   // [n_tiles] or null
};

// Pixel of lane `lane` in step `s` of chunk `c`: tile 2 s + (lane >> 5) of the
// chunk, pixel (lane & 7, (lane >> 3) & 3) of the tile.
struct StepPixel {
  int32_t tile;
  int32_t idx;   // y w + x, or -1 outside the frame / tile range
  uint32_t m;    // material id, 0xFFFF outside
};

__device__ __forceinline__ StepPixel step_pixel(const ClassifyArgs &a, int chunk, int s, int lane) {
  StepPixel p;
  p.tile = chunk * kTilesPerChunk + 2 * s + (lane >> 5);
  const int q = lane & 31;
  const int tx = p.tile % a.tw, ty = p.tile / a.tw;
  const int x = tx * 8 + (q & 7), y = ty * 4 + (q >> 3);
  const bool in = p.tile < a.n_tiles && x < a.w && y < a.h;
  p.idx = in ? y * a.w + x : -1;
  p.m = in ? (uint32_t)a.mat[p.idx] : 0xFFFFu;
  return p;
}

// Steps are taken kPrefetch at a time: their material ids are loaded first,
// so that one wait covers all of them instead of one load latency per step.
constexpr int kPrefetch = 8;

// Kind of the pixel's tile (0 simple, 1 other) and the tile's class
// (0 no neural pixel, 1 simple, 2 mixed or sparse), from the 32 lanes of
// its half of the wavefront.
__device__ __forceinline__ void tile_kind(bool valid, uint32_t m, int lane, int &kind, int &cls) {
  const uint64_t vb = __ballot(valid);
  const int n = __popcll((vb >> (lane & 32)) & 0xFFFFFFFFull);
  uint32_t mn = valid ? m : 0xFFFFFFFFu, mx = valid ? m : 0u;
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor((int)mn, o, 32));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 32));
  }
  const bool simple = n > 16 && mn == mx;
  kind = simple ? 0 : 1;
  cls = n == 0 ? 0 : (simple ? 1 : 2);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Pass 1: per chunk and key, the number of valid pixels. LDS: 2 n_mats ints.
__global__ __launch_bounds__(64) void classify_count_kernel(ClassifyArgs a) {
  extern __shared__ int32_t cnt[];
  const int lane = threadIdx.x;
  const int chunk = blockIdx.x;
  const int n_keys = 2 * a.n_mats;
  for (int k = lane; k < n_keys; k += 64) cnt[k] = 0;
  __syncthreads();
  for (int s0 = 0; s0 < kTilesPerChunk / 2; s0 += kPrefetch) {
    StepPixel ps[kPrefetch];
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) ps[i] = step_pixel(a, chunk, s0 + i, lane);
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) {
      const StepPixel p = ps[i];
      const bool valid = p.m < (uint32_t)a.n_mats;
      int kind, cls;
      tile_kind(valid, p.m, lane, kind, cls);
      if (a.tile_class && (lane & 31) == 0 && p.tile < a.n_tiles) a.tile_class[p.tile] = (uint8_t)cls;
      const int key = valid ? 2 * (int)p.m + kind : -1;
      uint64_t pending = __ballot(valid);
      while (pending) {
        const int leader = __builtin_ctzll(pending);
        const int k = __builtin_amdgcn_readlane(key, leader);
        const uint64_t same = __ballot(key == k);
        if (lane == 0) cnt[k] += __popcll(same);
        pending &= ~same;
      }
    }
  }
  __syncthreads();
  for (int k = lane; k < n_keys; k += 64) a.counts[(int64_t)k * a.n_chunks + chunk] = cnt[k];
}

// Pass 2a: one workgroup per key, exclusive prefix over chunks (in place),
// total per key.
__global__ __launch_bounds__(kScanThreads) void classify_scan_chunks_kernel(ClassifyArgs a) {
  __shared__ int32_t part[kScanThreads];
  const int key = blockIdx.x;
  int32_t *c = a.counts + (int64_t)key * a.n_chunks;
  const int per = (a.n_chunks + kScanThreads - 1) / kScanThreads;
  const int b0 = threadIdx.x * per, b1 = min(b0 + per, a.n_chunks);
  int32_t sum = 0;
  for (int i = b0; i < b1; ++i) sum += c[i];
  part[threadIdx.x] = sum;
  __syncthreads();
  // inclusive scan of the partial sums (Hillis-Steele)
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const int32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int32_t run = part[threadIdx.x] - sum;
  for (int i = b0; i < b1; ++i) {
    const int32_t v = c[i];
    c[i] = run;
    run += v;
  }
  if (threadIdx.x == kScanThreads - 1) a.totals[key] = part[kScanThreads - 1];
}

// Pass 2b: one workgroup, exclusive prefix over materials of their totals.
__global__ __launch_bounds__(kScanThreads) void classify_scan_materials_kernel(ClassifyArgs a) {
  __shared__ int32_t part[kScanThreads];
  const int per = (a.n_mats + kScanThreads - 1) / kScanThreads;
  const int m0 = threadIdx.x * per, m1 = min(m0 + per, a.n_mats);
  int32_t sum = 0;
  for (int m = m0; m < m1; ++m) sum += a.totals[2 * m] + a.totals[2 * m + 1];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const int32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int32_t run = part[threadIdx.x] - sum;
  for (int m = m0; m < m1; ++m) {
    a.mat_offsets[m] = run;
    a.mat_simple[m] = a.totals[2 * m];
    run += a.totals[2 * m] + a.totals[2 * m + 1];
  }
  if (threadIdx.x == kScanThreads - 1) a.mat_offsets[a.n_mats] = part[kScanThreads - 1];
}

// Pass 3: write every valid pixel's index at its place. LDS: 2 n_mats ints
// (the running position of each key inside this chunk's share).
__global__ __launch_bounds__(64) void classify_write_kernel(ClassifyArgs a) {
  extern __shared__ int32_t run[];
  const int lane = threadIdx.x;
  const int chunk = blockIdx.x;
  const int n_keys = 2 * a.n_mats;
  for (int k = lane; k < n_keys; k += 64) {
    const int m = k >> 1;
    run[k] = a.mat_offsets[m] + ((k & 1) ? a.totals[k - 1] : 0) + a.counts[(int64_t)k * a.n_chunks + chunk];
  }
  __syncthreads();
  for (int s0 = 0; s0 < kTilesPerChunk / 2; s0 += kPrefetch) {
    StepPixel ps[kPrefetch];
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) ps[i] = step_pixel(a, chunk, s0 + i, lane);
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) {
      const StepPixel p = ps[i];
      const bool valid = p.m < (uint32_t)a.n_mats;
      int kind, cls;
      tile_kind(valid, p.m, lane, kind, cls);
      const int key = valid ? 2 * (int)p.m + kind : -1;
      uint64_t pending = __ballot(valid);
      while (pending) {
        const int leader = __builtin_ctzll(pending);
        const int k = __builtin_amdgcn_readlane(key, leader);
        const uint64_t same = __ballot(key == k);
        const int base = run[k];
        if (key == k) a.list[base + (int)lanes_below(same)] = p.idx;
        // every lane has read run[k] before lane 0 moves it (one wavefront,
        // LDS operations complete in order)
        if (lane == 0) run[k] = base + __popcll(same);
        pending &= ~same;
      }
    }
  }
}

__global__ void gather_uv_kernel(const float2 *uv_image, const int32_t *list, int64_t n, float2 *uv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) uv[i] = uv_image[list[i]];
}

template <class T>
__global__ void scatter_rows_kernel(const T *rows, const int32_t *list, int64_t n, int c, T *image) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t i = e / c;
  image[(int64_t)list[i] * c + (e - i * c)] = rows[e];
}

}  // namespace

int classify_chunks(int w, int h) {
  const int64_t tiles = (int64_t)((w + 7) / 8) * ((h + 3) / 4);
  return (int)((tiles + kTilesPerChunk - 1) / kTilesPerChunk);
}

size_t classify_workspace_bytes(int w, int h, int n_mats) {
  const size_t keys = 2 * (size_t)n_mats;
  return (keys * (size_t)classify_chunks(w, h) + keys) * sizeof(int32_t);
}

hipError_t launch_classify(const uint16_t *mat, int w, int h, int n_mats, int32_t *list, int32_t *mat_offsets,
                           int32_t *mat_simple, uint8_t *tile_class, void *workspace, hipStream_t st) {
  ClassifyArgs a{};
  a.mat = mat;
  a.w = w;
  a.h = h;
  a.tw = (w + 7) / 8;
  a.n_tiles = a.tw * ((h + 3) / 4);
  a.n_chunks = classify_chunks(w, h);
  a.n_mats = n_mats;
  a.counts = static_cast<int32_t *>(workspace);
  a.totals = a.counts + (int64_t)2 * n_mats * a.n_chunks;
  a.mat_offsets = mat_offsets;
  a.mat_simple = mat_simple;
  a.list = list;
  a.tile_class = tile_class;
  const size_t lds = 2 * (size_t)n_mats * sizeof(int32_t);
  hipLaunchKernelGGL(classify_count_kernel, dim3(a.n_chunks), dim3(64), lds, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(classify_scan_chunks_kernel, dim3(2 * n_mats), dim3(kScanThreads), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(classify_scan_materials_kernel, dim3(1), dim3(kScanThreads), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(classify_write_kernel, dim3(a.n_chunks), dim3(64), lds, st, a);
  return hipGetLastError();
}

size_t classify_scratch_bytes() { return kClassifyScratchBytes; }

// Device address of this GPU's copy of `scratch`. In host code the array's
// name only stands in for the symbol; its device address is looked up once
// per device (with that device current) and kept.
hipError_t classify_scratch(void **ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_gather_uv(const float *uv_image, const int32_t *list, int64_t n, float *uv, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_uv_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<const float2 *>(uv_image), list, n, reinterpret_cast<float2 *>(uv));
  return hipGetLastError();
}

hipError_t launch_scatter_rows(const void *rows, const int32_t *list, int64_t n, int c, int elem_bytes, void *image,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t total = n * c;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (elem_bytes == 4)
    hipLaunchKernelGGL(scatter_rows_kernel<float>, grid, dim3(256), 0, st, static_cast<const float *>(rows), list,
                       n, c, static_cast<float *>(image));
  else
    hipLaunchKernelGGL(scatter_rows_kernel<uint16_t>, grid, dim3(256), 0, st, static_cast<const uint16_t *>(rows),
                       list, n, c, static_cast<uint16_t *>(image));
  return hipGetLastError();
}

}  // namespace ntc
