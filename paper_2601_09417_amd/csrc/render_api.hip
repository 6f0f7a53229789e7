// Host side of the renderer: batch planning, workspace layout and the launch sequence of
// vbm_render_fwd / vbm_render_bwd.
//
// Forward: project every (view, Gaussian) item -> stable compaction of visible items with their
// float32 depth bits as keys -> radix sort of those 31-bit keys (items in depth order, all views
// together, item index as the tie-break) -> exclusive scan of tile counts in that order -> emit
// (tile, item) pairs in depth/item order -> stable radix sort by global tile id alone, which leaves
// every tile's list (a tile belongs to one view) in (depth, item) order -> tile ranges -> tile
// launch order, longest lists first -> compositing.  Sorting items by depth once and then pairs by
// tile only needs ceil(tile_bits / digit) passes over the pairs instead of a full 64-bit
// (tile, depth) key sort.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace vbm {

__global__ void k_project(const DevView*, int, vbm_gaussians_c, float*, uint32_t*, float4*, float4*, float*,
                          uint32_t*, uint4*, unsigned long long*, unsigned long long*, uint32_t);
__global__ void k_compact_visible(const DevView*, const uint32_t*, const float*, const uint32_t*, uint32_t*,
                                  uint32_t*);
__global__ void k_gather_bins(const uint32_t*, const uint4*, const uint32_t*, int64_t, uint32_t*, uint4*);
__global__ void k_emit(const DevView*, int, const uint32_t*, const uint32_t*, const uint4*,
                       const float4*, const float4*, const unsigned long long*, int, uint32_t*, int64_t, int64_t,
                       uint32_t*, uint32_t*);
__global__ void k_ranges(const uint32_t*, const uint32_t*, int64_t, uint2*);
__global__ void k_status(const uint32_t*, int32_t*);
__global__ void k_tile_keys(const uint2*, int64_t, uint32_t*, uint32_t*);
__global__ void k_project_bwd(const DevView*, int, const DevScene*, int, vbm_gaussians_c, float*, const float4*,
                              int64_t, const uint32_t*, vbm_gaussians, int, int64_t);
vbm_status launch_composite_fwd(int tile, int lds_batch, const DevView* views, int n_views, int64_t n_tiles,
                                const uint2* ranges, const uint32_t* tile_order, const uint32_t* pair_item,
                                int64_t n_pairs, uint32_t* pair_marked, const float* coef, const float* blue,
                                int64_t n_items, float* image, float* final_T, int32_t* n_contrib,
                                unsigned long long* stats, hipStream_t s);
vbm_status launch_composite_bwd(int tile, int lds_batch, const DevView* views, int n_views, int64_t n_tiles,
                                const uint2* ranges, const uint32_t* tile_order, const uint32_t* pair_item,
                                const uint32_t* pair_marked, const float* coef, const float* blue,
                                const float* final_T, const int32_t* n_contrib, const float* dL_dimg, float* grad2d,
                                int64_t n_items, unsigned long long* stats, hipStream_t s);

namespace {

enum Region {
  R_COUNTERS = VBM_REGION_COUNTERS,
  R_DEPTH = VBM_REGION_ITEM_DEPTH,
  R_BIN = VBM_REGION_ITEM_RECT,   // uint4 [n_items]: the projection's bin entries (see vbm.h)
  R_NTILES = VBM_REGION_ITEM_NTILES,
  R_REC = VBM_REGION_ITEM_REC,
  R_BLUE = VBM_REGION_ITEM_BLUE,
  R_PTILE = VBM_REGION_PAIR_TILE,
  R_PITEM = VBM_REGION_PAIR_ITEM,
  R_RANGES = VBM_REGION_RANGES,
  R_GRAD2D = VBM_REGION_GRAD2D,
  R_VKEYS = 10,
  R_VKEYS_ALT = 11,
  R_VVALS = 12,
  R_VVALS_ALT = 13,
  R_POFFS = 14,
  R_PTILE_ALT = 15,
  R_PITEM_ALT = 16,
  R_SCRATCH = 17,
  R_VISFLAG = 18,
  R_COEF = VBM_REGION_ITEM_COEF,
  R_UNUSED20 = 20,
  R_TORDER = 21,   // uint32 [4][n_tiles]: sort keys, tiles, and the sorted keys and tiles (the launch order)
  R_WORDS = 22,    // uint64 [ballot_words(n_items)]: large rectangles' reached-tile ballots
  R_SBIN = 23,     // uint4 [n_items]: the visible items' bin entries in depth order
  R_COUNT = 24
};
static_assert(R_COUNT <= VBM_WS_REGIONS, "plan has room for every region");

// Capacity of the ballot-word buffer: one word per four items (at 1M Gaussians x 8 views the large
// rectangles need about 0.4M words of the 2M); rectangles that find it full are tested again by
// the emission instead.
int64_t ballot_words(int64_t n_items) { return n_items / 4 > 1024 ? n_items / 4 : 1024; }

int ceil_log2(int64_t x) {
  int b = 0;
  while ((static_cast<int64_t>(1) << b) < x) ++b;
  return b;
}

void layout(vbm_plan* p) {
  const int64_t I = p->n_items > 0 ? p->n_items : 1;
  const int64_t P = p->pair_capacity;
  const int64_t NT = p->n_tiles;
  size_t sz[R_COUNT];
  sz[R_COUNTERS] = 16 * 4;
  sz[R_DEPTH] = I * 4;
  sz[R_BIN] = I * 16;
  sz[R_NTILES] = I * 4;
  sz[R_REC] = I * 16;
  sz[R_BLUE] = I * 4;
  sz[R_PTILE] = P * 4;
  sz[R_PITEM] = P * 4;
  sz[R_RANGES] = NT * 8;
  sz[R_GRAD2D] = 16 * I * 4;
  sz[R_VKEYS] = I * 4;
  sz[R_VKEYS_ALT] = I * 4;
  sz[R_VVALS] = I * 4;
  sz[R_VVALS_ALT] = I * 4;
  sz[R_POFFS] = I * 4;
  sz[R_PTILE_ALT] = P * 4;
  sz[R_PITEM_ALT] = P * 4;
  size_t scr = scan_scratch_bytes(I);
  const size_t r1 = radix_scratch_bytes(I, 8);
  const size_t r2 = radix_scratch_bytes(P, p->sort_bits);
  if (r1 > scr) scr = r1;
  if (r2 > scr) scr = r2;
  const size_t r3 = radix_scratch_bytes(NT, 8);
  if (r3 > scr) scr = r3;
  sz[R_SCRATCH] = scr;
  sz[R_VISFLAG] = I * 4;
  sz[R_COEF] = I * 32;
  sz[R_UNUSED20] = 0;
  sz[R_TORDER] = 4 * NT * 4;
  sz[R_WORDS] = 8 * ballot_words(I);
  sz[R_SBIN] = I * 16;
  size_t off = 0;
  for (int r = 0; r < VBM_WS_REGIONS; ++r) {
    p->region_offset[r] = 0;
    p->region_bytes[r] = 0;
  }
  for (int r = 0; r < R_COUNT; ++r) {
    off = align_up(off, 256);
    p->region_offset[r] = off;
    p->region_bytes[r] = sz[r];
    off += sz[r];
  }
  p->ws_bytes = align_up(off, 256);
}

template <class T>
T* region(const vbm_plan* p, void* ws, int r) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + p->region_offset[r]);
}

// Launch order of the tiles for compositing (written by the forward): the sorted-tiles quarter of
// the order region.
uint32_t* tile_order(const vbm_plan* p, void* ws) { return region<uint32_t>(p, ws, R_TORDER) + 3 * p->n_tiles; }

vbm_status check_gaussians(const vbm_gaussians_c& g, const vbm_plan* p, const char* who) {
  if (!g.means || !g.scales || !g.quats || !g.opacity || !g.rgb) {
    set_error("%s: null Gaussian pointer", who);
    return VBM_ERR_INVALID;
  }
  if (g.stride < p->n_gaussians) {
    set_error("%s: Gaussian stride %lld < %lld Gaussians", who, static_cast<long long>(g.stride),
              static_cast<long long>(p->n_gaussians));
    return VBM_ERR_INVALID;
  }
  return VBM_OK;
}

vbm_status check_plan(const vbm_plan* p, const void* views, void* ws, size_t ws_bytes, const char* who) {
  if (!p || !views || !ws) {
    set_error("%s: null plan, view table or workspace", who);
    return VBM_ERR_INVALID;
  }
  if (p->tile != 8 && p->tile != 16 && p->tile != 32) {
    set_error("%s: plan has unsupported tile %d", who, p->tile);
    return VBM_ERR_UNSUPPORTED;
  }
  if (ws_bytes < p->ws_bytes) {
    set_error("%s: workspace %zu < %zu bytes", who, ws_bytes, p->ws_bytes);
    return VBM_ERR_WORKSPACE;
  }
  return VBM_OK;
}

int grid_cap(int64_t n, int64_t cap) {
  int64_t b = ceil_div(n > 0 ? n : 1, 256);
  return static_cast<int>(b < cap ? b : cap);
}

// Events recorded around the compositing launches when set (see vbm_profile_events).
hipEvent_t g_prof[4] = {nullptr, nullptr, nullptr, nullptr};
unsigned long long* g_stats = nullptr;  // device [4]: fwd evaluated, fwd contributing, bwd evaluated, bwd contributing

vbm_status record(int which, hipStream_t s) {
  if (!g_prof[which]) return VBM_OK;
  return hip_check(hipEventRecord(g_prof[which], s), "profile event record");
}

}  // namespace
}  // namespace vbm

using namespace vbm;

extern "C" vbm_status vbm_plan_make(const vbm_view* views, int32_t n_views, const int64_t* scene_offsets,
                                    int32_t n_scenes, const vbm_schedule* sch, vbm_plan* plan, void* table) {
  if (!views || !scene_offsets || !sch || !plan) {
    set_error("vbm_plan_make: null argument");
    return VBM_ERR_INVALID;
  }
  if (n_views < 1 || n_views > 4096 || n_scenes < 1 || n_scenes > 4096) {
    set_error("vbm_plan_make: need 1..4096 views and scenes");
    return VBM_ERR_INVALID;
  }
  if (sch->tile != 8 && sch->tile != 16 && sch->tile != 32) {
    set_error("vbm_plan_make: tile must be 8, 16 or 32 (got %d)", sch->tile);
    return VBM_ERR_UNSUPPORTED;
  }
  auto lds_ok = [&](int32_t b) { return b == 0 || ((b == 32 || b == 64) && sch->tile <= 16); };
  if (!lds_ok(sch->lds_batch) || !lds_ok(sch->lds_batch_bwd)) {
    set_error("vbm_plan_make: lds_batch and lds_batch_bwd must be 0, or 32 or 64 with 8x8 or 16x16 tiles");
    return VBM_ERR_UNSUPPORTED;
  }
  if (sch->sort_bits < 4 || sch->sort_bits > 8) {
    set_error("vbm_plan_make: sort_bits must be 4..8");
    return VBM_ERR_INVALID;
  }
  if (sch->pair_capacity < 1 || sch->pair_capacity >= (static_cast<int64_t>(1) << 30)) {
    set_error("vbm_plan_make: pair_capacity must be in [1, 2^30)");
    return VBM_ERR_INVALID;
  }
  if (sch->mode != VBM_MODE_BATCHED && sch->mode != VBM_MODE_EXACT) {
    set_error("vbm_plan_make: unknown mode %d", sch->mode);
    return VBM_ERR_INVALID;
  }
  if (scene_offsets[0] != 0) {
    set_error("vbm_plan_make: scene_offsets[0] must be 0");
    return VBM_ERR_INVALID;
  }
  for (int s = 0; s < n_scenes; ++s)
    if (scene_offsets[s + 1] < scene_offsets[s]) {
      set_error("vbm_plan_make: scene_offsets must not decrease");
      return VBM_ERR_INVALID;
    }
  std::memset(plan, 0, sizeof(*plan));
  plan->n_views = n_views;
  plan->n_scenes = n_scenes;
  plan->tile = sch->tile;
  plan->mode = sch->mode;
  plan->sort_bits = sch->sort_bits;
  plan->lds_batch = sch->lds_batch;
  plan->lds_batch_bwd = sch->lds_batch_bwd;
  plan->pair_capacity = sch->pair_capacity;
  plan->n_gaussians = scene_offsets[n_scenes];
  std::vector<DevView> dv(n_views);
  int64_t items = 0, tiles = 0, pixels = 0;
  for (int v = 0; v < n_views; ++v) {
    const vbm_view& in = views[v];
    if (in.scene < 0 || in.scene >= n_scenes) {
      set_error("vbm_plan_make: view %d references scene %d of %d", v, in.scene, n_scenes);
      return VBM_ERR_INVALID;
    }
    if (in.width < 1 || in.height < 1 || in.width > 16384 || in.height > 16384) {
      set_error("vbm_plan_make: view %d has size %dx%d", v, in.width, in.height);
      return VBM_ERR_INVALID;
    }
    if (!(in.fx > 0.0f) || !(in.fy > 0.0f) || !(in.near_plane > 0.0f) || !std::isfinite(in.cx) ||
        !std::isfinite(in.cy)) {
      set_error("vbm_plan_make: view %d has invalid intrinsics or near plane", v);
      return VBM_ERR_INVALID;
    }
    DevView& d = dv[v];
    std::memset(&d, 0, sizeof(d));
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) d.R[r * 3 + c] = in.viewmat[r * 4 + c];
      d.t[r] = in.viewmat[r * 4 + 3];
    }
    d.fx = in.fx;
    d.fy = in.fy;
    d.cx = in.cx;
    d.cy = in.cy;
    d.near_plane = in.near_plane;
    for (int c = 0; c < 3; ++c) d.bg[c] = in.bg[c];
    d.width = in.width;
    d.height = in.height;
    // same float32 operations as the projection's specification
    d.lim_x = 1.3f * ((0.5f * static_cast<float>(in.width)) / in.fx);
    d.lim_y = 1.3f * ((0.5f * static_cast<float>(in.height)) / in.fy);
    d.tiles_x = static_cast<int32_t>(ceil_div(in.width, sch->tile));
    d.tiles_y = static_cast<int32_t>(ceil_div(in.height, sch->tile));
    const int64_t ng = scene_offsets[in.scene + 1] - scene_offsets[in.scene];
    d.item_offset = static_cast<int32_t>(items);
    d.gauss_offset = static_cast<int32_t>(scene_offsets[in.scene]);
    d.n_gauss = static_cast<int32_t>(ng);
    d.tile_offset = static_cast<int32_t>(tiles);
    d.pixel_offset = static_cast<int32_t>(pixels);
    d.scene = in.scene;
    items += ng;
    tiles += static_cast<int64_t>(d.tiles_x) * d.tiles_y;
    pixels += static_cast<int64_t>(in.width) * in.height;
    // Items are addressed by 32-bit byte offsets into their 32-byte compositing records.
    if (items >= (static_cast<int64_t>(1) << 27) || tiles >= (static_cast<int64_t>(1) << 31) ||
        3 * pixels >= (static_cast<int64_t>(1) << 31) || plan->n_gaussians >= (static_cast<int64_t>(1) << 31)) {
      set_error("vbm_plan_make: batch exceeds 2^27 items or 2^31 tiles, Gaussians or image values");
      return VBM_ERR_INVALID;
    }
  }
  plan->n_items = items;
  plan->n_tiles = tiles;
  plan->n_pixels = pixels;
  plan->tile_key_bits = ceil_log2(tiles);
  plan->view_table_bytes = sizeof(DevView) * n_views + sizeof(DevScene) * n_scenes;
  layout(plan);
  if (table) {
    std::memcpy(table, dv.data(), sizeof(DevView) * n_views);
    DevScene* sc = reinterpret_cast<DevScene*>(static_cast<char*>(table) + sizeof(DevView) * n_views);
    for (int s = 0; s < n_scenes; ++s) {
      sc[s].gauss_offset = static_cast<int32_t>(scene_offsets[s]);
      sc[s].n_gauss = static_cast<int32_t>(scene_offsets[s + 1] - scene_offsets[s]);
    }
  }
  return VBM_OK;
}

extern "C" vbm_status vbm_render_fwd(const vbm_plan* p, const void* view_table, vbm_gaussians_c g, float* image,
                                     float* final_T, int32_t* n_contrib, int32_t* status, void* ws, size_t ws_bytes,
                                     void* stream) {
  VBM_TRY(check_plan(p, view_table, ws, ws_bytes, "vbm_render_fwd"));
  VBM_TRY(check_gaussians(g, p, "vbm_render_fwd"));
  if (!image || !final_T || !n_contrib || !status) {
    set_error("vbm_render_fwd: null output");
    return VBM_ERR_INVALID;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevView* views = static_cast<const DevView*>(view_table);
  const int64_t I = p->n_items;
  const int64_t cap = p->pair_capacity;
  uint32_t* counters = region<uint32_t>(p, ws, R_COUNTERS);
  float* depth = region<float>(p, ws, R_DEPTH);
  uint32_t* ntiles = region<uint32_t>(p, ws, R_NTILES);
  float4* rec = region<float4>(p, ws, R_REC);
  float4* coef = region<float4>(p, ws, R_COEF);
  float* blue = region<float>(p, ws, R_BLUE);
  uint32_t* visflag = region<uint32_t>(p, ws, R_VISFLAG);
  uint32_t* vk[2] = {region<uint32_t>(p, ws, R_VKEYS), region<uint32_t>(p, ws, R_VKEYS_ALT)};
  uint32_t* vv[2] = {region<uint32_t>(p, ws, R_VVALS), region<uint32_t>(p, ws, R_VVALS_ALT)};
  uint32_t* poffs = region<uint32_t>(p, ws, R_POFFS);
  uint32_t* pt[2] = {region<uint32_t>(p, ws, R_PTILE), region<uint32_t>(p, ws, R_PTILE_ALT)};
  uint32_t* pi[2] = {region<uint32_t>(p, ws, R_PITEM), region<uint32_t>(p, ws, R_PITEM_ALT)};
  uint2* ranges = region<uint2>(p, ws, R_RANGES);
  void* scratch = region<void>(p, ws, R_SCRATCH);

  VBM_TRY(fill_u32(counters, 0u, 16, s));
  // grid.x covers the largest scene (bounded by the total Gaussian count); grid.y is the view
  const int gx = static_cast<int>(ceil_div(p->n_gaussians > 0 ? p->n_gaussians : 1, 256));
  if (I > 0) {
    hipLaunchKernelGGL(k_project, dim3(gx, p->n_views), dim3(256), 0, s, views, p->tile, g, depth, ntiles, rec,
                       coef, blue, visflag, region<uint4>(p, ws, R_BIN),
                       reinterpret_cast<unsigned long long*>(counters + 4), region<unsigned long long>(p, ws, R_WORDS),
                       static_cast<uint32_t>(ballot_words(I)));
    VBM_LAUNCH_CHECK("project");
    VBM_TRY(scan_exclusive_u32(visflag, visflag, I, nullptr, &counters[0], scratch, s));
    // Visible items sorted by depth alone, all views together: a visible item's depth is positive,
    // so its float32 bits order like the depths and the sign bit is 0 (31 key bits, 4 passes).
    // Items of different views interleave, but every tile belongs to one view and the stable tile
    // sort that follows keeps this order inside each tile: (tile, depth, item).
    constexpr int kDepthKeyBits = 31;
    const int item_passes = static_cast<int>(ceil_div(kDepthKeyBits, 8));
    const int first = item_passes % 2;  // compact into the buffer that leaves the sorted data in slot 0
    hipLaunchKernelGGL(k_compact_visible, dim3(gx, p->n_views), dim3(256), 0, s, views, ntiles, depth, visflag,
                       vk[first], vv[first]);
    VBM_LAUNCH_CHECK("compact_visible");
    bool in_alt = false;
    VBM_TRY(radix_sort_pairs<uint32_t>(vk[first], vv[first], vk[1 - first], vv[1 - first], I, &counters[0],
                                       kDepthKeyBits, 8, scratch, s, &in_alt));
    hipLaunchKernelGGL(k_gather_bins, dim3(grid_cap(I, 8192)), dim3(256), 0, s, vv[0], region<uint4>(p, ws, R_BIN),
                       counters, I, poffs, region<uint4>(p, ws, R_SBIN));
    VBM_LAUNCH_CHECK("gather_bins");
    VBM_TRY(scan_exclusive_u32(poffs, poffs, I, &counters[0], &counters[1], scratch, s));
  }
  int64_t emit_grid_n = I;
  int64_t pair_n = cap;
  const uint32_t* pair_n_dev = &counters[1];
  if (p->mode == VBM_MODE_EXACT) {
    uint32_t host_counts[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(host_counts, counters, sizeof(host_counts), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_check(e, "vbm_render_fwd: count readback");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_check(e, "vbm_render_fwd: stream sync");
    emit_grid_n = host_counts[0];
    pair_n = host_counts[1] < cap ? host_counts[1] : cap;
    pair_n_dev = nullptr;
  }
  const int tile_passes = static_cast<int>(ceil_div(p->tile_key_bits, p->sort_bits));
  const int pfirst = tile_passes % 2;
  if (I > 0 && emit_grid_n > 0) {
    hipLaunchKernelGGL(k_emit, dim3(grid_cap(emit_grid_n, 16384)), dim3(256), 0, s, views, p->n_views, vv[0], poffs,
                       region<uint4>(p, ws, R_SBIN), rec, coef, region<unsigned long long>(p, ws, R_WORDS), p->tile,
                       counters, I, cap, pt[pfirst], pi[pfirst]);
    VBM_LAUNCH_CHECK("emit");
  }
  if (pair_n > 0) {
    bool in_alt = false;
    VBM_TRY(radix_sort_pairs<uint32_t>(pt[pfirst], pi[pfirst], pt[1 - pfirst], pi[1 - pfirst], pair_n, pair_n_dev,
                                       p->tile_key_bits, p->sort_bits, scratch, s, &in_alt));
  }
  VBM_TRY(fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * p->n_tiles, s));
  if (pair_n > 0) {
    hipLaunchKernelGGL(k_ranges, dim3(grid_cap(pair_n, 16384)), dim3(256), 0, s, pt[0], counters, cap, ranges);
    VBM_LAUNCH_CHECK("ranges");
  }
  if (p->n_tiles > 0) {
    // Longest lists first: one stable 8-bit pass over coarse length keys.
    const int64_t NT = p->n_tiles;
    uint32_t* tk = region<uint32_t>(p, ws, R_TORDER);
    hipLaunchKernelGGL(k_tile_keys, dim3(ceil_div(NT, 256)), dim3(256), 0, s, ranges, NT, tk, tk + NT);
    VBM_LAUNCH_CHECK("tile_keys");
    bool in_alt = false;   // one pass, so the sorted tiles land in the last quarter
    VBM_TRY(radix_sort_pairs<uint32_t>(tk, tk + NT, tk + 2 * NT, tk + 3 * NT, NT, nullptr, 8, 8, scratch, s, &in_alt));
  }
  VBM_TRY(record(0, s));
  // the sorted pair values stay in pi[0]; the forward's marked copy goes to the idle ping-pong buffer
  VBM_TRY(launch_composite_fwd(p->tile, p->lds_batch, views, p->n_views, p->n_tiles, ranges, tile_order(p, ws), pi[0],
                               cap, pi[1],
                               reinterpret_cast<const float*>(coef), blue, I, image, final_T, n_contrib, g_stats, s));
  VBM_TRY(record(1, s));
  hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, s, counters, status);
  VBM_LAUNCH_CHECK("status");
  return VBM_OK;
}

extern "C" vbm_status vbm_render_bwd(const vbm_plan* p, const void* view_table, vbm_gaussians_c g,
                                     const float* dL_dimg, const float* final_T, const int32_t* n_contrib,
                                     vbm_gaussians grads, int32_t accumulate, void* ws, size_t ws_bytes,
                                     void* stream) {
  VBM_TRY(check_plan(p, view_table, ws, ws_bytes, "vbm_render_bwd"));
  VBM_TRY(check_gaussians(g, p, "vbm_render_bwd"));
  if (!dL_dimg || !final_T || !n_contrib || !grads.means || !grads.scales || !grads.quats || !grads.opacity ||
      !grads.rgb) {
    set_error("vbm_render_bwd: null argument");
    return VBM_ERR_INVALID;
  }
  if (grads.stride < p->n_gaussians) {
    set_error("vbm_render_bwd: gradient stride too small");
    return VBM_ERR_INVALID;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevView* views = static_cast<const DevView*>(view_table);
  const DevScene* scenes =
      reinterpret_cast<const DevScene*>(static_cast<const char*>(view_table) + sizeof(DevView) * p->n_views);
  const int64_t I = p->n_items;
  float* grad2d = region<float>(p, ws, R_GRAD2D);
  VBM_TRY(fill_u32(reinterpret_cast<uint32_t*>(grad2d), 0u, 16 * I, s));
  VBM_TRY(record(2, s));
  VBM_TRY(launch_composite_bwd(p->tile, p->lds_batch_bwd, views, p->n_views, p->n_tiles, region<uint2>(p, ws, R_RANGES),
                               tile_order(p, ws),
                               region<uint32_t>(p, ws, R_PITEM), region<uint32_t>(p, ws, R_PITEM_ALT),
                               region<float>(p, ws, R_COEF), region<float>(p, ws, R_BLUE), final_T, n_contrib, dL_dimg,
                               grad2d, I, g_stats ? g_stats + 2 : nullptr, s));
  VBM_TRY(record(3, s));
  if (p->n_gaussians > 0) {
    hipLaunchKernelGGL(k_project_bwd, dim3(ceil_div(p->n_gaussians, 256)), dim3(256), 0, s, views, p->n_views, scenes,
                       p->n_scenes, g, grad2d, region<float4>(p, ws, R_REC), I, region<uint32_t>(p, ws, R_NTILES),
                       grads, accumulate,
                       p->n_gaussians);
    VBM_LAUNCH_CHECK("project_bwd");
  }
  return VBM_OK;
}

extern "C" vbm_status vbm_profile_events(void* fwd_begin, void* fwd_end, void* bwd_begin, void* bwd_end) {
  vbm::g_prof[0] = static_cast<hipEvent_t>(fwd_begin);
  vbm::g_prof[1] = static_cast<hipEvent_t>(fwd_end);
  vbm::g_prof[2] = static_cast<hipEvent_t>(bwd_begin);
  vbm::g_prof[3] = static_cast<hipEvent_t>(bwd_end);
  return VBM_OK;
}

extern "C" vbm_status vbm_profile_counters(void* dev_counters) {
  vbm::g_stats = static_cast<unsigned long long*>(dev_counters);
  return VBM_OK;
}
