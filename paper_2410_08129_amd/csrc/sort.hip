// Stable LSD radix sort of the (tile key, Gaussian index) instances and the
// per-tile ranges (Sec. 4.3: plain tile-id keys, no depth sort). The same
// pass kernel sorts the Gaussians by the view depth of their means for
// sorted blending (the 3DGS order that the paper's "w/o per-pixel HT"
// configuration blends in, Sec. 4.3, Table splat_eval).
//
// One launch per 8-bit digit. Each workgroup takes a chunk of 4096 keys (in
// ticket order), ranks them stably inside each 64-lane wave with ballots
// (lanes whose digits match, counted below the lane), combines the four
// waves in LDS, publishes its digit counts for the decoupled look-back over
// earlier chunks, and reorders the chunk by digit in LDS. The look-back gives
// each digit's global offset; the chunk then writes its LDS copy in order,
// so consecutive lanes store consecutive addresses of one digit's run. The
// global digit histograms were accumulated by the preprocess launch while it
// emitted the keys, so a pass reads its keys and values once and writes them
// once.
#include "common.h"

namespace htgs {

constexpr int kSortWaves = kSortThreads / 64;

// What one sort pass works on: the item count (a device word, or a fixed
// number), the capacity beyond which nothing is sorted, the global digit
// histograms, look-back words and tickets of its passes, and the status
// bits that cancel a pass (a give-up of an earlier stage) or that a give-up
// of this pass sets.
struct SortJob {
  const unsigned long long *count;  // null: n_fixed items
  uint64_t n_fixed;
  int64_t capacity;
  const uint32_t *hist;             // [passes][256]
  uint32_t *look;                   // [passes][max_chunks][256]
  uint32_t *tickets;                // one per pass
  uint32_t *status;
  int64_t max_chunks;
  uint32_t cancel[4];               // per pass
  uint32_t spin[4];                 // per pass
  int32_t spin_limit;
};

template <typename KeyT>
__global__ void __launch_bounds__(kSortThreads) k_sort_pass(SortJob job, int pass, int nbits,
                                                             const KeyT *__restrict__ kin,
                                                             const uint32_t *__restrict__ vin,
                                                             KeyT *__restrict__ kout,
                                                             uint32_t *__restrict__ vout) {
  static_assert(kSortThreads == 256, "one thread per digit");
  __shared__ uint32_t s_wh[kSortWaves][256];  // per wave and digit: count, then local offset
  __shared__ uint32_t s_off[256];             // global position of local slot 0, per digit
  __shared__ uint32_t s_wsum[kSortWaves];
  __shared__ uint32_t s_csum[kSortWaves];
  __shared__ uint32_t s_ticket;
  __shared__ KeyT s_key[kSortChunk];
  __shared__ uint32_t s_val[kSortChunk];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned long long tot = job.count ? *job.count : job.n_fixed;
  // On overflow only part of the keys exist while the histograms count all
  // of them; after a give-up of the preprocess or an earlier pass the keys
  // (and their slots) are not the counted ones. Nothing is sorted then, and
  // the status word reports why. (A give-up inside this pass only moves
  // positions down within [0, I): every later launch sees its flag.)
  if (tot > (unsigned long long)job.capacity) return;
  if (ld_acq_u32(&job.status[0]) & job.cancel[pass]) return;
  const uint64_t I = tot;
  const uint64_t nchunks = (I + kSortChunk - 1) / kSortChunk;
  if (tid == 0) s_ticket = atomicAdd(&job.tickets[pass], 1u);
  for (int i = tid; i < kSortWaves * 256; i += kSortThreads) (&s_wh[0][0])[i] = 0u;

  // Exclusive scan of the global digit histogram of this pass.
  const uint32_t hv = job.hist[pass * 256 + tid];
  uint32_t x = hv;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_wsum[wave] = x;
  __syncthreads();
  uint32_t woff = 0;
  for (int k = 0; k < wave; ++k) woff += s_wsum[k];
  const uint32_t digit_excl = x + woff - hv;
  const uint64_t chunk = s_ticket;
  if (chunk >= nchunks) return;  // uniform over the workgroup

  const int shift = 8 * pass;
  const uint64_t cbase = chunk * kSortChunk;
  const uint64_t wbase = cbase + (uint64_t)wave * (64 * kSortItems);
  KeyT key[kSortItems];
  uint32_t val[kSortItems];
  uint32_t rank[kSortItems];
  const uint64_t lanemask_lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint64_t idx = wbase + (uint64_t)i * 64 + lane;
    const bool valid = idx < I;
    key[i] = valid ? kin[idx] : (KeyT)0;
    val[i] = valid ? vin[idx] : 0u;
  }
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint64_t idx = wbase + (uint64_t)i * 64 + lane;
    const bool valid = idx < I;
    const uint32_t d = ((uint32_t)key[i] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t lt = (uint32_t)__popcll(peers & lanemask_lt);
    uint32_t old = 0;
    if (valid) old = s_wh[wave][d];
    rank[i] = old + lt;
    // Lanes of one wave reach LDS in issue order, so the leader's update is
    // seen by the next item's reads without a barrier.
    if (valid && lt == 0) s_wh[wave][d] = old + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // Per digit (thread d): counts of the chunk, published at once for the
  // successors' look-back; the local start of each digit is the exclusive
  // scan of the counts over digits.
  const int d = tid;
  uint32_t cnt = 0;
#pragma unroll
  for (int k = 0; k < kSortWaves; ++k) cnt += s_wh[k][d];
  uint32_t *look = job.look + ((size_t)pass * (size_t)job.max_chunks) * 256;
  st_rel_u32(&look[chunk * 256 + d], (chunk == 0 ? kFlagP32 : kFlagA32) | cnt);
  uint32_t c = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(c, off, 64);
    if (lane >= off) c += y;
  }
  if (lane == 63) s_csum[wave] = c;
  __syncthreads();
  uint32_t local_start = c - cnt;
  for (int k = 0; k < wave; ++k) local_start += s_csum[k];
  {
    uint32_t run = local_start;
#pragma unroll
    for (int k = 0; k < kSortWaves; ++k) {
      const uint32_t v = s_wh[k][d];
      s_wh[k][d] = run;
      run += v;
    }
  }
  __syncthreads();

  // Reorder the chunk by digit in LDS.
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint64_t idx = wbase + (uint64_t)i * 64 + lane;
    if (idx < I) {
      const uint32_t dd = ((uint32_t)key[i] >> shift) & 255u;
      const uint32_t lp = s_wh[wave][dd] + rank[i];
      s_key[lp] = key[i];
      s_val[lp] = val[i];
    }
  }

  // Look-back over earlier chunks for this digit's global offset, reading
  // kLookWindow predecessors per round trip.
  uint32_t excl = 0;
  if (chunk > 0) {
    int64_t j = (int64_t)chunk - 1;
    int spins = 0;
    while (true) {
      if (spins > job.spin_limit) {  // give up (a negative limit: at once)
        atomicOr(&job.status[0], job.spin[pass]);
        break;
      }
      uint32_t sv[kLookWindow];
#pragma unroll
      for (int k = 0; k < kLookWindow; ++k)
        sv[k] = (j - k >= 0) ? ld_acq_u32(&look[(j - k) * 256 + d]) : 0u;
      int used = 0;
      bool done = false;
#pragma unroll
      for (int k = 0; k < kLookWindow; ++k) {
        if (done || used < k) continue;      // stop at the first P or unpublished word
        const uint32_t f = sv[k] >> 30;
        if (f == 0) continue;
        excl += sv[k] & kMask32;
        used = k + 1;
        done = (f == 2);
      }
      if (done) break;
      j -= used;
      if (used == 0) {
        ++spins;
        __builtin_amdgcn_s_sleep(1);
      }
    }
    st_rel_u32(&look[chunk * 256 + d], kFlagP32 | (excl + cnt));
  }
  // position of local slot p of digit d: digit_excl + excl + (p - local_start)
  s_off[d] = digit_excl + excl - local_start;
  __syncthreads();

  const uint64_t left = I - cbase;
  const int n_local = left < (uint64_t)kSortChunk ? (int)left : kSortChunk;
  for (int p = tid; p < n_local; p += kSortThreads) {
    const KeyT k = s_key[p];
    const uint32_t pos = s_off[((uint32_t)k >> shift) & 255u] + (uint32_t)p;
    kout[pos] = k;
    vout[pos] = s_val[p];
  }
}

// Per-tile [start, end): each thread takes 8 consecutive sorted keys (one
// or two 16-byte loads) plus the key before them, and marks the key changes.
template <typename KeyT>
__global__ void __launch_bounds__(256) k_ranges(Ws w, const KeyT *__restrict__ keys,
                                                 uint32_t total_tiles) {
  const unsigned long long tot = *w.total;
  // overflow or a give-up: the keys are not a sorted list, every tile stays empty
  if (tot > (unsigned long long)w.capacity || front_failed(w)) return;
  const uint64_t I = tot;
  const uint64_t ngroups = (I + 7) / 8;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t gi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < ngroups; gi += stride) {
    const uint64_t i0 = gi * 8;
    uint32_t k[8];
    if (i0 + 8 <= I) {
      if constexpr (sizeof(KeyT) == 2) {
        const uint4 t = *reinterpret_cast<const uint4 *>(keys + i0);
        const uint32_t u[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) { k[2 * j] = u[j] & 0xffffu; k[2 * j + 1] = u[j] >> 16; }
      } else {
        const uint4 a = *reinterpret_cast<const uint4 *>(keys + i0);
        const uint4 b = *reinterpret_cast<const uint4 *>(keys + i0 + 4);
        k[0] = a.x; k[1] = a.y; k[2] = a.z; k[3] = a.w; k[4] = b.x; k[5] = b.y; k[6] = b.z; k[7] = b.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) k[j] = (i0 + j < I) ? (uint32_t)keys[i0 + j] : 0u;
    }
    uint32_t prev = i0 > 0 ? (uint32_t)keys[i0 - 1] : 0xffffffffu;
    const uint32_t next = (i0 + 8 < I) ? (uint32_t)keys[i0 + 8] : 0xffffffffu;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint64_t i = i0 + j;
      if (i >= I) break;
      const uint32_t nk = (j < 7 && i + 1 < I) ? k[j + 1] : (j == 7 ? next : 0xffffffffu);
      if (k[j] < total_tiles) {
        if (i == 0 || k[j] != prev) w.ranges[k[j]].x = (uint32_t)i;
        if (i + 1 == I || k[j] != nk) w.ranges[k[j]].y = (uint32_t)(i + 1);
      }
      prev = k[j];
    }
  }
}

// Tiles in descending order of their instance count, by power-of-two
// buckets (bucket clz(count) - 1; empty tiles last). The order inside a
// bucket is arbitrary; it only decides which workgroup runs a tile first.
__device__ __forceinline__ uint32_t cost_bucket(uint2 r) {
  const uint32_t c = r.y - r.x;
  return c == 0 ? 31u : (uint32_t)__clz(c) - 1u;
}

// Counting sort of the tiles by bucket: each workgroup counts its tiles in
// LDS and adds one total per bucket to the global histogram; the placing
// pass reserves one run per (workgroup, bucket) with one atomic and fills
// it from LDS cursors.
__global__ void __launch_bounds__(256) k_tile_order_count(Ws w, int total_tiles) {
  __shared__ uint32_t s_cnt[32];
  if (threadIdx.x < 32) s_cnt[threadIdx.x] = 0u;
  __syncthreads();
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total_tiles; t += gridDim.x * blockDim.x)
    atomicAdd(&s_cnt[cost_bucket(w.ranges[t])], 1u);
  __syncthreads();
  if (threadIdx.x < 32 && s_cnt[threadIdx.x]) atomicAdd(&w.order_hist[threadIdx.x], s_cnt[threadIdx.x]);
}

__global__ void __launch_bounds__(256) k_tile_order_place(Ws w, int total_tiles) {
  __shared__ uint32_t s_base[32], s_cnt[32], s_run[32];
  if (threadIdx.x < 32) {
    uint32_t b = 0;
    for (uint32_t k = 0; k < threadIdx.x; ++k) b += w.order_hist[k];
    s_base[threadIdx.x] = b;
    s_cnt[threadIdx.x] = 0u;
  }
  __syncthreads();
  // this workgroup's tiles: same grid-stride set as the counting pass
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total_tiles; t += gridDim.x * blockDim.x)
    atomicAdd(&s_cnt[cost_bucket(w.ranges[t])], 1u);
  __syncthreads();
  if (threadIdx.x < 32) {
    const uint32_t c = s_cnt[threadIdx.x];
    s_run[threadIdx.x] = c ? s_base[threadIdx.x] + atomicAdd(&w.order_hist[32 + threadIdx.x], c) : 0u;
    s_cnt[threadIdx.x] = 0u;
  }
  __syncthreads();
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total_tiles; t += gridDim.x * blockDim.x) {
    const uint32_t b = cost_bucket(w.ranges[t]);
    w.order[s_run[b] + atomicAdd(&s_cnt[b], 1u)] = (uint32_t)t;
  }
}

hipError_t launch_tile_order(const Ws &w, int total_tiles, hipStream_t s) {
  int blocks = (total_tiles + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_tile_order_count, dim3(blocks), dim3(256), 0, s, w, total_tiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_order_place, dim3(blocks), dim3(256), 0, s, w, total_tiles);
  return hipGetLastError();
}

template <typename KeyT>
static hipError_t sort_impl(const Ws &w, hipStream_t s) {
  SortJob job{};
  job.count = w.total;
  job.capacity = w.capacity;
  job.hist = w.hist;
  job.look = w.sort_look;
  job.tickets = w.status + kTicketSort;
  job.status = w.status;
  job.max_chunks = w.max_chunks;
  job.spin_limit = w.spin_limit;
  for (int p = 0; p < 4; ++p) {
    job.cancel[p] = spin_bits_before_sort(p);
    job.spin[p] = (uint32_t)ST_SPIN | ((uint32_t)ST_SPIN_SORT0 << p);
  }
  const int blocks = (int)(w.max_chunks > 0 ? w.max_chunks : 1);
  for (int p = 0; p < w.passes; ++p) {
    const int nbits = (w.key_bits - 8 * p) < 8 ? (w.key_bits - 8 * p) : 8;
    const KeyT *kin = reinterpret_cast<const KeyT *>(w.keys[p & 1]);
    KeyT *kout = reinterpret_cast<KeyT *>(w.keys[(p + 1) & 1]);
    hipLaunchKernelGGL(k_sort_pass<KeyT>, dim3(blocks), dim3(kSortThreads), 0, s, job, p, nbits,
                       kin, w.vals[p & 1], kout, w.vals[(p + 1) & 1]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Sort key of sorted blending: the view depth of the mean, the third row of
// the world-to-camera transform applied to it in float64 (x, y and z terms
// in that order, then the translation; the products of float32 values are
// exact) and rounded to float32, as an unsigned integer of the same order
// (-0 taken as +0). Each workgroup also counts its keys' four digits.
__global__ void __launch_bounds__(256) k_depth_keys(const float *__restrict__ means, int64_t n,
                                                     float r0, float r1, float r2, float t,
                                                     uint32_t *__restrict__ keys,
                                                     uint32_t *__restrict__ idx,
                                                     uint32_t *__restrict__ hist) {
  __shared__ uint32_t s_hist[4][256];
  for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) (&s_hist[0][0])[i] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += stride) {
    const double z = (((double)r0 * (double)means[3 * g] + (double)r1 * (double)means[3 * g + 1]) +
                      (double)r2 * (double)means[3 * g + 2]) + (double)t;
    float zf = (float)z;
    if (zf == 0.0f) zf = 0.0f;
    const uint32_t u = __float_as_uint(zf);
    const uint32_t key = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    keys[g] = key;
    idx[g] = (uint32_t)g;
#pragma unroll
    for (int p = 0; p < 4; ++p) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) {
    const uint32_t c = (&s_hist[0][0])[i];
    if (c) atomicAdd(&hist[i], c);
  }
}

// The Gaussians front to back by the view depth of their means, ties by
// index (a stable sort of the index order): depth keys, then four 8-bit
// passes; the order ends in w.dvals[0].
hipError_t launch_depth_sort(const Ws &w, const float *means, int64_t n, const float *w2c,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_depth_keys, dim3(blocks), dim3(256), 0, s, means, n, w2c[8], w2c[9],
                     w2c[10], w2c[11], w.dkeys[0], w.dvals[0], w.dhist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  SortJob job{};
  job.count = nullptr;
  job.n_fixed = (uint64_t)n;
  job.capacity = n;
  job.hist = w.dhist;
  job.look = w.dlook;
  job.tickets = w.status + kDsortTicket;
  job.status = w.status;
  job.max_chunks = w.dmax_chunks;
  job.spin_limit = w.spin_limit;
  for (int p = 0; p < 4; ++p) {
    job.cancel[p] = spin_bits_before_dsort(p);
    job.spin[p] = (uint32_t)ST_SPIN | ((uint32_t)ST_SPIN_DSORT0 << p);
  }
  const int sblocks = (int)((n + kSortChunk - 1) / kSortChunk);
  for (int p = 0; p < 4; ++p) {
    hipLaunchKernelGGL(k_sort_pass<uint32_t>, dim3(sblocks), dim3(kSortThreads), 0, s, job, p, 8,
                       w.dkeys[p & 1], w.dvals[p & 1], w.dkeys[(p + 1) & 1],
                       w.dvals[(p + 1) & 1]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename KeyT>
static hipError_t ranges_impl(const Ws &w, int total_tiles, hipStream_t s) {
  const KeyT *sorted = reinterpret_cast<const KeyT *>(w.keys[w.passes & 1]);
  int rb = (int)((w.capacity + 8 * 256 - 1) / (8 * 256));
  if (rb < 1) rb = 1;
  if (rb > 8192) rb = 8192;
  hipLaunchKernelGGL(k_ranges<KeyT>, dim3(rb), dim3(256), 0, s, w, sorted, (uint32_t)total_tiles);
  return hipGetLastError();
}

hipError_t launch_sort_passes(const Ws &w, hipStream_t s) {
  if (w.capacity == 0) return hipSuccess;
  return w.key16 ? sort_impl<uint16_t>(w, s) : sort_impl<uint32_t>(w, s);
}

hipError_t launch_ranges(const Ws &w, int total_tiles, hipStream_t s) {
  if (w.capacity == 0) return hipSuccess;
  return w.key16 ? ranges_impl<uint16_t>(w, total_tiles, s)
                 : ranges_impl<uint32_t>(w, total_tiles, s);
}

}  // namespace htgs
