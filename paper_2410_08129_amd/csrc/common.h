// Internal definitions shared by the HIP kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace htgs {

constexpr int kMaxViews = 16;
constexpr int kRecFloats = 32;      // per (view, Gaussian) raster record
constexpr int kPartialFloats = 16;  // per-instance backward partials (64 bytes)
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortChunk = kSortThreads * kSortItems;
constexpr int kPreThreads = 256;

// Raster record of one Gaussian in one view (float32). The Pluecker
// direction d and moment m of the ray through a pixel are affine in the
// pixel's offset from a reference pixel (ix, iy) inside the splat's
// footprint: d = D0 + dx Du + dy Dv, m = M0 + dx Mu + dy Mv, with dx, dy
// the integer pixel offsets. Centring keeps the float32 evaluation of m
// accurate where rho is small.
enum RecField {
  R_D0 = 0, R_DU = 3, R_DV = 6, R_M0 = 9, R_MU = 12, R_MV = 15,
  R_R3 = 18,    // third view row of M T (scaled axes' z components)
  R_MUZ = 21,   // view depth of the mean
  R_O = 22,     // opacity
  R_RC = 23,    // rho_c (squared cutoff radius)
  R_RGB = 24,   // colour (3)
  R_FLAGS = 27, // bit c set: colour channel c was clamped at 0 (also in Ws::cflags)
  R_IX = 28, R_IY = 29,  // reference pixel, int32 bit patterns
  R_BB0 = 30,   // covered pixel rect: x0 | y0 << 16
  R_BB1 = 31    //                     x1 | y1 << 16 (inclusive)
};

// Per-instance backward partials, summed over one tile's pixels p of one
// (view, Gaussian): the moments sum_p w(p) (1, dx, dy, dx^2, dx dy, dy^2)
// of the weights w = dL/d(d) / d and dL/d(m) / m (the loss gradient
// w.r.t. the Pluecker vectors is w(p) times the vector), with (dx, dy) the
// pixel's offset from the record's reference pixel (ix, iy) (the covered
// pixel nearest the centre of the splat's screen box); then
// dL/do and dL/d(rgb). Moments about one origin add up over the tiles, and
// the preprocess backward turns the sums into coefficient gradients once.
enum PartialField {
  P_MD = 0, P_MM = 6, P_O = 12, P_C = 13
};

struct ViewParams {
  float w2c[12];        // row-major [R|t]
  float fx, fy, cx, cy;
  double cam_pos[3];    // camera centre -R^-1 t (computed on the host in float64)
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  int32_t tile_base;    // first global tile id of this view
  float z_near;
  int64_t state_off;    // float offset of this view's state block
  float *out_rgb;       // [3,H,W]
  const float *grad_rgb;
};

struct ViewSet {
  int32_t n;
  int32_t total_tiles;
  ViewParams v[kMaxViews];
};

struct KCfg {
  int64_t n;
  int32_t K;
  int32_t sh_degree;
  float tau_alpha, tau_core, alpha_max;
  float bg[3];
  int32_t tile_w, tile_h;
  int32_t batch_mult;   // records staged per forward thread and batch (1 or 2)
  int32_t cost_order;   // raster workgroups take tiles in descending-cost order
  int32_t grad_overwrite;  // preprocess backward stores gradients instead of adding
  int32_t tile_cull;       // drop rect tiles that no fragment can reach (rects of <= 64 tiles)
  int32_t persistent;      // raster workgroups pull tiles from an atomic queue
  int32_t no_tail;         // forward leaves the tail out (inference)
  int32_t baked;           // inputs hold scales, unit quaternions and opacities
  int32_t sorted;          // alpha blending in mean-depth order with an early stop
  float tau_T;             // sorted blending stops before T falls below this
};

struct GaussPtrs {
  const float *means, *log_scales, *quats, *logits, *sh;
  const float *filter_var;   // 3D filter variance per Gaussian, or null
};

struct GradPtrs {
  float *means, *log_scales, *quats, *logits, *sh;
  float *mean_grad_stat, *visible_count;   // densification sums, or null
};

// Ws::cflags bit: the Gaussian's screen box holds a pixel centre of the view.
constexpr uint32_t kCflagVisible = 8u;

// Device addresses inside the caller's workspace.
struct Ws {
  uint32_t *status;            // [kStatusWords]: flags, raster queues (see below)
  unsigned long long *total;   // instance count (64-bit)
  unsigned long long *frags;   // fragments counted by the forward raster (spread, below)
  unsigned long long *frags_bwd;  // fragments counted by the backward raster (spread)
  unsigned long long *pp_total;  // per preprocess workgroup: its instance total, then its first slot
  uint32_t *hist;              // [kHistCopies][4][256] digit histograms (summed when read)
  uint32_t *sort_cnt;          // [passes][256][chunk_stride]: per-chunk digit counts, then
                               // the global start of each (digit, chunk) run
  uint2 *ranges;               // [total_tiles] (start, end)
  uint32_t *order_hist;        // [2][32] cost-bucket counts and cursors
  uint32_t *order;             // [total_tiles] tiles by descending instance count
  float *records;              // [views][n][32]
  int4 *rects;                 // [views][n] tile rect (tx0, ty0, tx1, ty1), empty if tx0 > tx1
  uint4 *tslots;               // [views][n] tile-slot descriptor (see below)
  uint32_t *refpix;            // [views][n] the record's reference pixel ix | iy << 16
  uint8_t *cflags;             // [views][n] bit c < 3: colour channel c was clamped at 0;
                               // kCflagVisible: the pixel rect is not empty
  void *keys[2];
  uint32_t *vals[2];
  float *partials;             // [capacity][24]
  // Sorted blending: the Gaussians' mean-depth sort keys, sorted (key,
  // index) pairs (ping-pong; the final index buffer is the order the
  // preprocess walks), its digit histograms and per-chunk counts.
  uint32_t *dkeys[2];
  uint32_t *dvals[2];
  uint32_t *dhist;             // [kHistCopies][4][256]
  uint32_t *dcnt;              // [4][256][dchunk_stride]
  const uint32_t *perm;        // Gaussians front to back (null: index order)
  int64_t dchunk_stride;
  int64_t capacity;
  int64_t chunk_stride;        // words per digit row of sort_cnt (>= chunks of capacity)
  int32_t key_bits, passes, key16;
  int32_t final_buf;           // which of keys/vals holds the sorted lists
};

// Forward state values per pixel: K ids, K alphas, K list positions, K rgb
// triples, T, sum alpha, sum alpha rgb (3), prod (1 - alpha).
__host__ __device__ constexpr int state_values(int K) { return 6 * K + 6; }
// Sorted blending's state per pixel: T after the last blended fragment, the
// blended colour sum (3), the list position after the last blended
// fragment, the number of blended fragments, the Gaussian the early stop
// left out (-1: none).
constexpr int kSortedStateValues = 7;

// Digit histograms: kHistCopies copies, added to by workgroup
// blockIdx % kHistCopies and summed by the sort's scan. With one copy the
// emit launch's end-of-workgroup adds (one per non-empty digit, ~24 per
// workgroup) queued on 16 cache lines and set its length (87 us at 1080p).
constexpr int kHistCopies = 64;
__device__ __forceinline__ uint32_t *hist_copy(uint32_t *hist) {
  return hist + (blockIdx.x % kHistCopies) * (4 * 256);
}

// LDS digit histogram of one wave's keys, in C copies of kHistPadWords
// words (copy c at c * kHistPadWords, so that the copies of a digit lie in
// different banks): for digits of at most two bits, one ballot per digit
// value and one add each; otherwise one add per lane into copy lane % C.
// Lanes of one wave that add to one address are served one after another,
// and tile keys often share their high digits across a wave (one add per
// lane on one copy made the high passes' counting many times slower; a
// test for a wave whose keys all share one digit cost more than it saved).
// Called by all lanes of the wave.
constexpr int kHistLaneCopies = 4, kHistPadWords = 257;
constexpr int kHistWords = kHistLaneCopies * kHistPadWords;
template <int C = kHistLaneCopies>
__device__ __forceinline__ void wave_hist_add(uint32_t *h, uint32_t d, bool valid, int nbits) {
  const uint64_t vm = __ballot(valid);
  if (vm == 0ull) return;
  const int lane = __lane_id();
  const int lead = (int)__builtin_ctzll(vm);
  if (nbits <= 2) {
    for (uint32_t v = 0; v < (1u << nbits); ++v) {
      const uint32_t c = (uint32_t)__popcll(__ballot(valid && d == v));
      if (lane == lead && c) atomicAdd(&h[v], c);
    }
    return;
  }
  if (valid) atomicAdd(&h[(lane % C) * kHistPadWords + d], 1u);
}
// Digit d of a histogram written by wave_hist_add<C>.
template <int C = kHistLaneCopies>
__device__ __forceinline__ uint32_t hist_total(const uint32_t *h, int d) {
  uint32_t t = 0;
#pragma unroll
  for (int c = 0; c < C; ++c) t += h[c * kHistPadWords + d];
  return t;
}
// Width of sort pass p's digit for keys of key_bits bits.
__host__ __device__ __forceinline__ int pass_bits(int key_bits, int p) {
  const int r = key_bits - 8 * p;
  return r < 8 ? r : 8;
}

// Fragment counters: kCounterSpread words, each in a 128-byte line of its
// own, added to by workgroup blockIdx % kCounterSpread and summed when
// read. With one word, the raster's tens of thousands of workgroups queued
// their end-of-tile atomics on one address (the 8x8 backward ran ~35%
// slower with one atomic per workgroup).
constexpr int kCounterSpread = 64;
constexpr int kCounterStride = 16;   // 64-bit words per 128-byte line
__device__ __forceinline__ void count_add(unsigned long long *ctr, unsigned long long v) {
  atomicAdd(ctr + (blockIdx.x % kCounterSpread) * kCounterStride, v);
}

// Status word: ST_OVERFLOW, more instances than the workspace holds (no
// workgroup of any launch waits for another, so nothing else can fail).
enum StatusBits : uint32_t { ST_OVERFLOW = 1u };
constexpr uint32_t kStatusPublic = ST_OVERFLOW;
// Status words (512 bytes, four 128-byte cache lines). The flags word has a
// line of its own: every workgroup of the later stages reads it. [0] flags;
// [64..67] / [68..71] the raster queues.
constexpr int kStatusWords = 128;
// outputs of the front end are unusable: overflow
__device__ __forceinline__ bool front_failed(const Ws &w) {
  return (__hip_atomic_load(&w.status[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
          ST_OVERFLOW) != 0u;
}
// status words of the persistent raster queues (16-byte aligned, cleared
// before each raster launch)
constexpr int kQueueFwd = 64, kQueueBwd = 68;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Instances of one (view, Gaussian): the rect's tiles, or the surviving
// ones when a tile mask is set.
// Tile-slot descriptor of one (view, Gaussian): x = first instance slot
// (offset of the Gaussian plus the counts of its earlier views), y = tile
// rect origin and width packed as tx0 | ty0 << 10 | width << 20, (z, w) =
// the 64-bit mask of surviving tiles of the rect (row-major bits, 0 = all).
__device__ __forceinline__ unsigned long long tslot_mask(uint4 d) {
  return (unsigned long long)d.z | ((unsigned long long)d.w << 32);
}

__device__ __forceinline__ int tile_count(int4 r, unsigned long long mask) {
  if (r.x > r.z || r.y > r.w) return 0;
  return mask ? __popcll(mask) : (r.z - r.x + 1) * (r.w - r.y + 1);
}

// Position of tile idx (row-major in the rect) among the instances of its
// (view, Gaussian).
__device__ __forceinline__ uint32_t tile_rank(int idx, unsigned long long mask) {
  return mask ? (uint32_t)__popcll(mask & ((1ull << idx) - 1ull)) : (uint32_t)idx;
}

__device__ __forceinline__ uint32_t tslot_slot(uint4 d, int tx, int ty) {
  const int x0 = (int)(d.y & 1023u), y0 = (int)((d.y >> 10) & 1023u), wdt = (int)(d.y >> 20);
  return d.x + tile_rank((ty - y0) * wdt + (tx - x0), tslot_mask(d));
}

// Tile coverage rule shared by the forward and backward launchers: tile ids
// are handed out so that consecutive workgroups on one XCD (workgroups are
// dealt round-robin over the 8 XCDs) work on a contiguous band of tiles.
__device__ __forceinline__ int xcd_tile(int block, int total_tiles) {
  const int per = (total_tiles + 7) >> 3;
  return (block & 7) * per + (block >> 3);
}

__device__ __forceinline__ int view_of_tile(const ViewSet &vs, int t) {
  int v = 0;
  for (int k = 1; k < vs.n; ++k) v = (t >= vs.v[k].tile_base) ? k : v;
  return v;
}

}  // namespace htgs
