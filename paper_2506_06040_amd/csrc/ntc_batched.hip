// Many materials in one persistent launch.
//
// The paper groups the pixels of a frame by MLP so that a workgroup always
// runs a single weight matrix on its matrix engines (Sec. 4), building
// per-MLP tile lists with a classification pass (Alg. 1). Here the grouping
// is done once on the host: each material's pixels are cut into work items
// of whole 64-pixel tiles, items are assigned to persistent waves by
// longest-processing-time-first bin packing on an estimated cost, and each
// wave's list is ordered by (MLP shape, material) so that a wave loads a
// material's weights into registers once per run of items. The launch
// itself has no queue, counter or atomic: every wave walks its own list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <queue>
#include <vector>

#include "ntc_device.hpp"
#include "ntc_internal.hpp"
#include "ntc_mfma_tile.hpp"

namespace ntc {

// 64-pixel tiles per span of the batched walk. One kernel holds every
// shape, so a longer span raises the register spills of all of them; it
// pays only for the 16- and 32-wide networks read in order (2% on the
// 64-material batch; with the 64-wide 3-layer ones and the indexed reads as
// well, 8.5% slower).
template <int HID, bool IDX>
constexpr int batch_span_tiles() {
  return (HID <= 32 && !IDX) ? NTC_SPAN_TILES_SMALL : NTC_SPAN_TILES;
}

template <int HID, int NL, int VEC4, bool IDX>
__device__ __forceinline__ void run_material(const BatchMaterial &M, const BatchItem *items, int it0, int it1,
                                             f32x4 *stage, f32x4 *bias, f32x4 *ltab) {
  constexpr int ST = batch_span_tiles<HID, IDX>();
  const DecodeArgs &a = M.a;
  const int lane = threadIdx.x;
  MfmaWeights<PrecF16, HID, NL> W;
  W.load(a.packed, a.lay, lane);
  // LDS tables of the previous material were last read by this wave's own
  // earlier instructions, which a single-wave workgroup completes in order
  BiasLds<HID, NL>::fill(bias, a.packed, a.lay, lane);
  LevelTab::fill(ltab, a.lat, lane);
  W.ready();
  __syncthreads();
  // walk spans of up to ST tiles inside each item; the uv of the next span
  // is prefetched
  auto item_end = [&](int it) {
    const int64_t t1 = items[it].first_tile + items[it].n_tiles;
    return t1 * 64 < a.n ? t1 * 64 : a.n;
  };
  SpanUv<ST> uvs;
  int it = it0;
  int64_t tile = items[it0].first_tile;
  uvs.template load_any<IDX>(a, tile * 64, item_end(it0));
  uvs.ready();
  while (it < it1) {
    const int64_t end_px = item_end(it);
    int nit = it;
    int64_t ntile = tile + ST;
    if (ntile >= items[it].first_tile + items[it].n_tiles) {
      ++nit;
      ntile = nit < it1 ? items[nit].first_tile : -1;
    }
    decode_span<PrecF16, HID, NL, ST, VEC4, IDX>(a, tile * 64, end_px, stage, bias, ltab, W, uvs,
                                            nit < it1 ? ntile * 64 : -1, nit < it1 ? item_end(nit) : 0);
    it = nit;
    tile = ntile;
  }
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NTC_WAVES_PER_SIMD, NTC_WAVES_PER_SIMD))) void decode_batched_kernel(const uint8_t *__restrict__ plan) {
  extern __shared__ f32x4 smem[];
  const BatchPlanHeader *h = reinterpret_cast<const BatchPlanHeader *>(plan);
  f32x4 *stage = smem;
  f32x4 *bias = smem + h->stage_cap;
  f32x4 *ltab = bias + BiasLds<64, 4>::kCount;
  const BatchMaterial *mats = reinterpret_cast<const BatchMaterial *>(plan + h->mats_off);
  const BatchItem *items = reinterpret_cast<const BatchItem *>(plan + h->items_off);
  const int32_t *start = reinterpret_cast<const int32_t *>(plan + h->wave_start_off);
  const int w = blockIdx.x;
  int it = start[w];
  const int end = start[w + 1];
  while (it < end) {
    const int m = items[it].mat;
    int run_end = it + 1;
    while (run_end < end && items[run_end].mat == m) ++run_end;
    const BatchMaterial &M = mats[m];
    const int oc = out_class(M.a.n_out);
#define NTC_RUN_O(HID, NL, IDX)                                                                        \
  (oc == kOut4 ? run_material<HID, NL, kOut4, IDX>(M, items, it, run_end, stage, bias, ltab)            \
               : (oc == kOut4x2 ? run_material<HID, NL, kOut4x2, IDX>(M, items, it, run_end, stage, bias, ltab) \
                                : run_material<HID, NL, kOutAny, IDX>(M, items, it, run_end, stage, bias, ltab)))
#define NTC_RUN(HID, NL) (M.a.pix ? NTC_RUN_O(HID, NL, true) : NTC_RUN_O(HID, NL, false))
    switch (M.shape_id) {
      case 0: NTC_RUN(16, 2); break;
      case 1: NTC_RUN(16, 3); break;
      case 2: NTC_RUN(16, 4); break;
      case 3: NTC_RUN(32, 2); break;
      case 4: NTC_RUN(32, 3); break;
      case 5: NTC_RUN(32, 4); break;
      case 6: NTC_RUN(64, 2); break;
      case 7: NTC_RUN(64, 3); break;
      case 8: NTC_RUN(64, 4); break;
      default: break;
    }
#undef NTC_RUN
#undef NTC_RUN_O
    it = run_end;
  }
}

// ---------------------------------------------------------------------------
// Host planner
// ---------------------------------------------------------------------------
int shape_id_of(int hid, int n_layers) {
  const int hi = hid == 16 ? 0 : (hid == 32 ? 1 : (hid == 64 ? 2 : -1));
  if (hi < 0 || n_layers < 2 || n_layers > 4) return -1;
  return 3 * hi + (n_layers - 2);
}

// Estimated cost of one 64-pixel tile: MFMA issue slots of the MLP plus a
// fixed share for sampling and staging.
static double tile_cost(int hid, int n_layers) {
  const int mt = hid / 16, kc = hid >= 32 ? hid / 32 : 1;
  const double mfma = 4.0 * (mt + (double)(n_layers - 2) * mt * kc + kc);
  return mfma + 12.0;
}

size_t plan_bytes(int n_mats, int64_t n_items, int n_waves) {
  size_t off = (sizeof(BatchPlanHeader) + 255) / 256 * 256;
  off += (size_t)n_mats * sizeof(BatchMaterial);
  off = (off + 255) / 256 * 256;
  off += (size_t)n_items * sizeof(BatchItem);
  off = (off + 255) / 256 * 256;
  off += (size_t)(n_waves + 1) * sizeof(int32_t);
  return (off + 255) / 256 * 256;
}

int64_t count_items(const int64_t *n_px, int n_mats, int item_tiles) {
  int64_t k = 0;
  for (int m = 0; m < n_mats; ++m) {
    const int64_t tiles = (n_px[m] + 63) / 64;
    k += (tiles + item_tiles - 1) / item_tiles;
  }
  return k;
}

int plan_waves(int64_t n_items, int n_cus, int waves_per_cu) {
  int64_t w = (int64_t)n_cus * waves_per_cu;
  if (w > n_items) w = n_items;
  return (int)(w < 1 ? 1 : w);
}

void build_plan(const BatchMaterial *mats, int n_mats, int item_tiles, int n_waves, int stage_cap, uint8_t *out,
                size_t bytes) {
  std::vector<BatchItem> items;
  std::vector<double> cost;
  for (int m = 0; m < n_mats; ++m) {
    const int64_t tiles = mats[m].a.n_tiles;
    const double c = tile_cost(mats[m].hid, mats[m].n_layers);
    for (int64_t t = 0; t < tiles; t += item_tiles) {
      BatchItem it;
      it.mat = m;
      it.shape_id = mats[m].shape_id;
      it.first_tile = t;
      it.n_tiles = std::min<int64_t>(item_tiles, tiles - t);
      items.push_back(it);
      cost.push_back(c * (double)it.n_tiles);
    }
  }
  // longest processing time first onto the least loaded wave
  std::vector<int64_t> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return cost[x] > cost[y]; });
  using Slot = std::pair<double, int>;
  std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
  for (int w = 0; w < n_waves; ++w) heap.push(Slot(0.0, w));
  std::vector<std::vector<int64_t>> per_wave(n_waves);
  for (int64_t i : order) {
    Slot s = heap.top();
    heap.pop();
    per_wave[s.second].push_back(i);
    s.first += cost[i];
    heap.push(s);
  }
  // within a wave: by shape, then material, then tile, so weights load once per run
  for (auto &v : per_wave)
    std::sort(v.begin(), v.end(), [&](int64_t x, int64_t y) {
      const BatchItem &p = items[x], &q = items[y];
      if (p.shape_id != q.shape_id) return p.shape_id < q.shape_id;
      if (p.mat != q.mat) return p.mat < q.mat;
      return p.first_tile < q.first_tile;
    });

  memset(out, 0, bytes);
  BatchPlanHeader h;
  memset(&h, 0, sizeof h);
  h.magic = kPlanMagic;
  h.version = kPlanVersion;
  h.n_mats = n_mats;
  h.n_items = (int32_t)items.size();
  h.n_waves = n_waves;
  h.stage_cap = stage_cap;
  size_t off = (sizeof(BatchPlanHeader) + 255) / 256 * 256;
  h.mats_off = off;
  off += (size_t)n_mats * sizeof(BatchMaterial);
  off = (off + 255) / 256 * 256;
  h.items_off = off;
  off += items.size() * sizeof(BatchItem);
  off = (off + 255) / 256 * 256;
  h.wave_start_off = off;
  off += (size_t)(n_waves + 1) * sizeof(int32_t);
  h.total_bytes = (off + 255) / 256 * 256;
  memcpy(out, &h, sizeof h);
  memcpy(out + h.mats_off, mats, (size_t)n_mats * sizeof(BatchMaterial));
  BatchItem *dst = reinterpret_cast<BatchItem *>(out + h.items_off);
  int32_t *start = reinterpret_cast<int32_t *>(out + h.wave_start_off);
  int32_t k = 0;
  for (int w = 0; w < n_waves; ++w) {
    start[w] = k;
    for (int64_t i : per_wave[w]) dst[k++] = items[i];
  }
  start[n_waves] = k;
}

hipError_t launch_decode_batched(const uint8_t *plan_dev, const BatchPlanHeader &h, hipStream_t st) {
  if (h.n_waves < 1) return hipSuccess;
  const size_t lds = (size_t)(h.stage_cap + BiasLds<64, 4>::kCount + LevelTab::kCount) * sizeof(f32x4);
  hipLaunchKernelGGL(decode_batched_kernel, dim3(h.n_waves), dim3(64), lds, st, plan_dev);
  return hipGetLastError();
}

}  // namespace ntc
