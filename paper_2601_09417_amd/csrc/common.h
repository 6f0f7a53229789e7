// Internal declarations shared by the libvbm translation units (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/vbm.h"

namespace vbm {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
vbm_status hip_check(hipError_t e, const char* what);
#define VBM_LAUNCH_CHECK(name)                                         \
  do {                                                                 \
    hipError_t _e = hipGetLastError();                                 \
    if (_e != hipSuccess) return ::vbm::hip_check(_e, name);           \
  } while (0)
#define VBM_TRY(expr)                                                  \
  do {                                                                 \
    vbm_status _s = (expr);                                            \
    if (_s != VBM_OK) return _s;                                       \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Bump allocator over a caller-provided workspace (sizing pass when base == nullptr).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// ------------------------------------------------------------------ device view table
// One record per view, written by vbm_plan_make on the host and read by every render kernel.
struct DevView {
  float R[9];            // world->camera rotation, row-major
  float t[3];
  float fx, fy, cx, cy;
  float near_plane;
  float bg[3];
  int32_t width, height, tiles_x, tiles_y;
  int32_t item_offset;   // first item of this view
  int32_t gauss_offset;  // first Gaussian of the view's scene
  int32_t n_gauss;       // Gaussians in the view's scene
  int32_t tile_offset;   // first global tile of this view
  int32_t pixel_offset;  // first pixel of this view
  int32_t scene;
  float lim_x, lim_y;    // FOV clamp of the projection Jacobian: 1.3 (0.5 W / fx), 1.3 (0.5 H / fy) in float32
};
static_assert(sizeof(DevView) % 16 == 0, "DevView must stay 16-byte aligned");

// Scene table appended after the views in the device view table.
struct DevScene {
  int32_t gauss_offset, n_gauss;
};

// ------------------------------------------------------------------ pair values
// A pair value holds the item id in bits 0..26 (the plan keeps items below 2^27) and a 4-bit mask
// of the tile's lane groups in bits 27..30.  With 16x16 tiles lane group k is pixel rows
// 4k .. 4k + 3 of the tile.  The emission sets the groups the footprint can reach (all four with
// other tiles), and the forward's marked copy the groups it evaluated.
constexpr int kItemBits = 27;
constexpr uint32_t kItemMask = (1u << kItemBits) - 1u;

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t popc_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// ------------------------------------------------------------------ arithmetic
// Correctly rounded float32 square root: the square root of the value in float64, rounded to
// float32.  Rounding twice cannot go wrong here because 53 >= 2 * 24 + 2 (the float64 result,
// even one unit off in its last place, never crosses a float32 rounding boundary); the float32
// square-root instruction alone is only accurate to one unit in the last place.
__device__ __forceinline__ float sqrt_rn_f32(float x) {
  return static_cast<float>(__dsqrt_rn(static_cast<double>(x)));
}

// ------------------------------------------------------------------ scan / sort primitives (scan_sort.hip)
// Exclusive prefix sum of n u32 values (n read from *n_dev when non-null, else n_max), with the
// total written to *total_dev.  Scratch from scan_scratch_bytes(n_max).
size_t scan_scratch_bytes(int64_t n_max);
vbm_status scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n_max, const uint32_t* n_dev,
                              uint32_t* total_dev, void* scratch, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs over key bits [0, end_bit) (end_bit <= 32), digit
// width 4..8 bits.  Passes ping-pong between (k0, v0) and (k1, v1); returns in *result_in_k1
// whether the sorted data ends in the second buffer.  The element count is read from *n_dev
// (<= n_max) when non-null.
size_t radix_scratch_bytes(int64_t n_max, int digit_bits);
template <class K>
vbm_status radix_sort_pairs(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t n_max, const uint32_t* n_dev,
                            int end_bit, int digit_bits, void* scratch, hipStream_t s, bool* result_in_k1);

// Device fill (used instead of memset nodes so every step stays capturable).
vbm_status fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);

}  // namespace vbm
