// Stable LSD radix sort of the (tile key, Gaussian index) instances and the
// per-tile ranges (Sec. 4.3: plain tile-id keys, no depth sort). The same
// passes sort the Gaussians by the view depth of their means for sorted
// blending (the 3DGS order that the paper's "w/o per-pixel HT"
// configuration blends in, Sec. 4.3, Table splat_eval).
//
// Three launches per 8-bit digit, none of whose workgroups waits for
// another. The keys are cut into chunks of 4096 in list order.
//   count:   each workgroup counts the digits of its chunk (LDS adds) and
//            stores the 256 counts into a digit-major table;
//   scan:    one workgroup per digit turns its row of chunk counts into the
//            global start of the digit's run from each chunk (the digit's
//            base is the sum of the smaller digits' totals, which the
//            preprocess counted while it emitted the keys);
//   scatter: each workgroup ranks its chunk again, stably within each wave
//            by ballots, reorders it by digit in LDS and writes every
//            digit's run at the start the scan gave it, so consecutive
//            lanes store consecutive addresses.
// A pass reads its keys twice and its values once and writes both once.
// The chunks are dealt to the eight XCDs (workgroups go round-robin over
// them) in contiguous ranges, so that the 32 chunks of a 128-byte line of a
// digit row are counted, and read back, on one XCD, and adjacent digit runs
// are written from one L2.
#include "common.h"

namespace htgs {

constexpr int kSortWaves = kSortThreads / 64;
constexpr int kScanItems = 8;   // chunk counts per thread per round of the scan

// What a sort works on: the item count (a device word, or a fixed number),
// the capacity beyond which nothing is sorted, the global digit histograms
// and the per-chunk count table (counts, then run starts).
struct SortJob {
  const unsigned long long *count;  // null: n_fixed items
  uint64_t n_fixed;
  int64_t capacity;
  const uint32_t *hist;             // [kHistCopies][4][256]
  uint32_t *cnt;                    // [passes][256][stride]: digit counts per chunk, then
                                    // the global start of each (digit, chunk) run
  int64_t stride;
};

// Items to sort, or false on overflow, when only part of the keys exist
// while the histograms count all of them (the status word reports it).
__device__ __forceinline__ bool sort_items(const SortJob &job, uint64_t &items) {
  const unsigned long long tot = job.count ? *job.count : job.n_fixed;
  if (tot > (unsigned long long)job.capacity) return false;
  items = tot;
  return true;
}

// Chunk of workgroup b < nchunks: XCD b mod 8 takes a contiguous range of
// the chunks (the first nchunks mod 8 XCDs one more).
__device__ __forceinline__ uint64_t chunk_of(uint64_t b, uint64_t nchunks) {
  const uint64_t q = nchunks >> 3, r = nchunks & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Lanes of the wave whose digit equals this lane's, among the lanes of
// `valid`: one ballot per digit bit (bits at and above nbits are zero in
// every key), and a lane differs from this one where a ballot bit differs
// from this lane's own bit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid, int nbits) {
  uint32_t xlo = 0u, xhi = 0u;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    if (b < nbits) {  // uniform
      const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);  // all ones where set
      const uint64_t bal = __ballot((int32_t)m < 0);
      xlo |= (uint32_t)bal ^ m;
      xhi |= (uint32_t)(bal >> 32) ^ m;
    }
  }
  return valid & ~(((uint64_t)xhi << 32) | (uint64_t)xlo);
}

__device__ __forceinline__ uint32_t digit_of(uint32_t key, int shift) { return (key >> shift) & 255u; }

// Inclusive sum over the lanes of a wave by DPP moves (shifts by 1, 2, 4, 8
// inside each row of 16 lanes, then the row ends broadcast to the rows
// after them); lanes whose source is outside receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ uint32_t wave_incl_add(uint32_t x) {
  x += dpp_u32<0x111, 0xf>(x);
  x += dpp_u32<0x112, 0xf>(x);
  x += dpp_u32<0x114, 0xf>(x);
  x += dpp_u32<0x118, 0xf>(x);
  x += dpp_u32<0x142, 0xa>(x);
  x += dpp_u32<0x143, 0xc>(x);
  return x;
}

// base[i] with a 32-bit byte offset (i * sizeof(T) < 2^32), so that the load
// takes the base in scalar registers and one 32-bit offset register
template <typename T>
__device__ __forceinline__ T load_at(const T *base, uint32_t i) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                      (uint32_t)(i * (uint32_t)sizeof(T)));
}

template <typename KeyT>
__global__ void __launch_bounds__(kSortThreads) k_sort_count(SortJob job, int pass, int nbits,
                                                              const KeyT *__restrict__ kin) {
  __shared__ uint32_t s_cnt[kHistWords];
  uint64_t I;
  if (!sort_items(job, I)) return;
  const uint64_t nchunks = (I + kSortChunk - 1) / kSortChunk;
  if (blockIdx.x >= nchunks) return;  // uniform over the workgroup
  const uint64_t chunk = chunk_of(blockIdx.x, nchunks);
  const uint64_t cbase = chunk * kSortChunk;
  const int tid = threadIdx.x;
  for (int i = tid; i < kHistWords; i += kSortThreads) s_cnt[i] = 0u;
  const int shift = 8 * pass;
  uint32_t dg[kSortItems];
  const bool whole = cbase + kSortChunk <= I;
  if (whole) {
    // the order of the keys does not matter here: 16-byte loads
    constexpr int kPer = 16 / (int)sizeof(KeyT);
    const uint4 *src = reinterpret_cast<const uint4 *>(kin + cbase);
#pragma unroll
    for (int j = 0; j < kSortItems / kPer; ++j) {
      const uint4 q = src[j * kSortThreads + tid];
      const uint32_t u[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        if constexpr (sizeof(KeyT) == 2) {
          dg[j * kPer + 2 * h] = digit_of(u[h] & 0xffffu, shift);
          dg[j * kPer + 2 * h + 1] = digit_of(u[h] >> 16, shift);
        } else {
          dg[j * kPer + h] = digit_of(u[h], shift);
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const uint64_t idx = cbase + (uint64_t)i * kSortThreads + tid;
      dg[i] = idx < I ? digit_of((uint32_t)kin[idx], shift) : 0u;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i)
    wave_hist_add(s_cnt, dg[i], whole || cbase + (uint64_t)i * kSortThreads + tid < I, nbits);
  __syncthreads();
  job.cnt[((size_t)pass * 256 + tid) * (size_t)job.stride + chunk] = hist_total(s_cnt, tid);
}

// One workgroup per digit: exclusive scan of its row of chunk counts, plus
// the digit's base, in place.
__global__ void __launch_bounds__(256) k_sort_scan(SortJob job, int pass) {
  __shared__ uint32_t s_wsum[4];
  __shared__ uint32_t s_base;
  uint64_t I;
  if (!sort_items(job, I)) return;
  const uint64_t nchunks = (I + kSortChunk - 1) / kSortChunk;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t dg = blockIdx.x;
  // base: the totals of the digits below this one
  uint32_t x = 0u;
  if (tid < (int)dg)
    for (int c = 0; c < kHistCopies; ++c) x += job.hist[(c * 4 + pass) * 256 + tid];
  const uint32_t wx = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_add(x), 63);
  if (lane == 0) s_wsum[wave] = wx;
  __syncthreads();
  if (tid == 0) s_base = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
  __syncthreads();
  uint32_t carry = s_base;
  uint32_t *row = job.cnt + ((size_t)pass * 256 + dg) * (size_t)job.stride;
  for (uint64_t c0 = 0; c0 < nchunks; c0 += 256 * kScanItems) {
    const uint64_t cb = c0 + (uint64_t)tid * kScanItems;
    uint32_t v[kScanItems];
    if (cb + kScanItems <= nchunks) {
      const uint4 a = *reinterpret_cast<const uint4 *>(row + cb);
      const uint4 b = *reinterpret_cast<const uint4 *>(row + cb + 4);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
      for (int j = 0; j < kScanItems; ++j) v[j] = cb + j < nchunks ? row[cb + j] : 0u;
    }
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) sum += v[j];
    const uint32_t inc = wave_incl_add(sum);
    __syncthreads();   // the previous round's readers of s_wsum are done
    if (lane == 63) s_wsum[wave] = inc;
    __syncthreads();
    uint32_t run = carry + inc - sum;
    for (int k = 0; k < wave; ++k) run += s_wsum[k];
    uint32_t out[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) { out[j] = run; run += v[j]; }
    if (cb + kScanItems <= nchunks) {
      *reinterpret_cast<uint4 *>(row + cb) = make_uint4(out[0], out[1], out[2], out[3]);
      *reinterpret_cast<uint4 *>(row + cb + 4) = make_uint4(out[4], out[5], out[6], out[7]);
    } else {
#pragma unroll
      for (int j = 0; j < kScanItems; ++j)
        if (cb + j < nchunks) row[cb + j] = out[j];
    }
    carry += s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
  }
}

template <typename KeyT>
__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(SortJob job, int pass, int nbits,
                                                                const KeyT *__restrict__ kin,
                                                                const uint32_t *__restrict__ vin,
                                                                KeyT *__restrict__ kout,
                                                                uint32_t *__restrict__ vout) {
  static_assert(kSortThreads == 256, "one thread per digit");
  __shared__ uint32_t s_wh[kSortWaves][256];  // per wave and digit: count, then local offset
  __shared__ uint32_t s_off[256];             // global position of local slot 0, per digit
  __shared__ uint32_t s_csum[kSortWaves];
  __shared__ KeyT s_key[kSortChunk];
  __shared__ uint32_t s_val[kSortChunk];

  uint64_t I;
  if (!sort_items(job, I)) return;
  const uint64_t nchunks = (I + kSortChunk - 1) / kSortChunk;
  if (blockIdx.x >= nchunks) return;  // uniform over the workgroup
  const uint64_t chunk = chunk_of(blockIdx.x, nchunks);
  const uint64_t cbase = chunk * kSortChunk;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // global start of this chunk's run of digit tid (from the scan)
  const uint32_t run_start = job.cnt[((size_t)pass * 256 + tid) * (size_t)job.stride + chunk];
  for (int i = tid; i < kSortWaves * 256; i += kSortThreads) (&s_wh[0][0])[i] = 0u;
  __syncthreads();

  // Items of the chunk: nv; lane l of wave w holds item w 1024 + 64 i + l
  // as its i-th (out-of-range lanes read the last item and take no part).
  const uint32_t nv = (I - cbase) < (uint64_t)kSortChunk ? (uint32_t)(I - cbase) : (uint32_t)kSortChunk;
  const int shift = 8 * pass;
  const uint32_t obase = (uint32_t)wave * (64 * kSortItems) + (uint32_t)lane;
  const KeyT *kc = kin + cbase;
  const uint32_t *vc = vin + cbase;
  uint32_t kx[kSortItems];   // the keys (widened)
  uint32_t val[kSortItems];
  uint32_t rank[kSortItems];
  const uint64_t lanemask_lt = (1ull << lane) - 1ull;
  // item i of this lane exists iff 64 i < rem
  const int rem = (int)nv - (int)obase;
  if (nv == (uint32_t)kSortChunk) {
    const KeyT *kp = kc + obase;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) kx[i] = kp[64 * i];
  } else {
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) kx[i] = load_at(kc, min(obase + 64u * i, nv - 1u));
  }
  // Rank: lanes with the same digit are ranked by lane; the lowest of them
  // adds their number to the wave's counter of the digit and hands the old
  // value to the others. One wave's LDS atomics are applied in issue order,
  // so item i's add is seen by item i + 1's and the ranks follow the list.
  // (all adds first, then the hand-overs, so that the adds' round trips
  // overlap)
  // The leader lane and the rank among the peers (6 bits each) wait in the
  // upper half of a 16-bit key's register, or in a register of their own.
  constexpr bool kPack = sizeof(KeyT) == 2;
  uint32_t lead[kPack ? 1 : kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const bool valid = 64 * i < rem;
    const uint32_t d = digit_of(kx[i], shift);
    const uint64_t peers = match_digit(d, __ballot(valid), nbits);
    const uint32_t lt = (uint32_t)__popcll(peers & lanemask_lt);
    uint32_t old = 0;
    if (valid && lt == 0) old = atomicAdd(&s_wh[wave][d], (uint32_t)__popcll(peers));
    rank[i] = old;
    const uint32_t ld = (valid ? (uint32_t)__builtin_ctzll(peers) : (uint32_t)lane) | (lt << 6);
    if constexpr (kPack) kx[i] |= ld << 16;
    else lead[i] = ld;
  }
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t ld = kPack ? kx[i] >> 16 : lead[kPack ? 0 : i];
    rank[i] = (uint32_t)__shfl(rank[i], (int)(ld & 63u), 64) + (ld >> 6);
  }
  __syncthreads();

  // Per digit (thread d): the chunk's count; the local start of each digit
  // is the exclusive scan of the counts over digits.
  const int d = tid;
  uint32_t cnt = 0;
#pragma unroll
  for (int k = 0; k < kSortWaves; ++k) cnt += s_wh[k][d];
  const uint32_t c = wave_incl_add(cnt);
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
  // position of local slot p of digit d: run_start + (p - local_start)
  s_off[d] = run_start - local_start;
  __syncthreads();

  // Reorder the chunk by digit in LDS (the values are loaded only now, which
  // keeps the ranking's register count down).
  // (an opaque copy of the keys: otherwise the compiler keeps every item's
  // LDS address of the ranking live until here)
  if (nv == (uint32_t)kSortChunk) {
    const uint32_t *vp = vc + obase;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) val[i] = vp[64 * i];
  } else {
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) val[i] = load_at(vc, min(obase + 64u * i, nv - 1u));
  }
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    if (64 * i < rem) {
      uint32_t kk = kPack ? (kx[i] & 0xffffu) : kx[i];
      asm volatile("" : "+v"(kk));
      const uint32_t lp = s_wh[wave][digit_of(kk, shift)] + rank[i];
      s_key[lp] = (KeyT)kk;
      s_val[lp] = val[i];
    }
  }
  __syncthreads();

  for (int p = tid; p < (int)nv; p += kSortThreads) {
    const KeyT k = s_key[p];
    const uint32_t pos = s_off[digit_of((uint32_t)k, shift)] + (uint32_t)p;
    if (pos < I) {  // always, when the counts match the emitted keys
      kout[pos] = k;
      vout[pos] = s_val[p];
    }
  }
}

// The three launches of each pass; blocks: the largest chunk count the
// item count can reach.
template <typename KeyT>
static hipError_t sort_passes(const SortJob &job, int passes, int key_bits, int64_t blocks,
                              void *const *keys, uint32_t *const *vals, hipStream_t s) {
  if (blocks < 1) blocks = 1;
  for (int p = 0; p < passes; ++p) {
    const int nbits = (key_bits - 8 * p) < 8 ? (key_bits - 8 * p) : 8;
    const KeyT *kin = reinterpret_cast<const KeyT *>(keys[p & 1]);
    KeyT *kout = reinterpret_cast<KeyT *>(keys[(p + 1) & 1]);
    hipLaunchKernelGGL(k_sort_count<KeyT>, dim3((uint32_t)blocks), dim3(kSortThreads), 0, s, job, p,
                       nbits, kin);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_scan, dim3(256), dim3(256), 0, s, job, p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_scatter<KeyT>, dim3((uint32_t)blocks), dim3(kSortThreads), 0, s, job,
                       p, nbits, kin, vals[p & 1], kout, vals[(p + 1) & 1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Per-tile [start, end): each thread takes 8 consecutive sorted keys (one
// or two 16-byte loads) plus the key before them, and marks the key changes.
template <typename KeyT>
__global__ void __launch_bounds__(256) k_ranges(Ws w, const KeyT *__restrict__ keys,
                                                 uint32_t total_tiles) {
  const unsigned long long tot = *w.total;
  // overflow: the keys are not a sorted list, every tile stays empty
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
  job.cnt = w.sort_cnt;
  job.stride = w.chunk_stride;
  return sort_passes<KeyT>(job, w.passes, w.key_bits, (w.capacity + kSortChunk - 1) / kSortChunk,
                           w.keys, w.vals, s);
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
  __shared__ uint32_t s_hist[4][kHistWords];
  for (int i = threadIdx.x; i < 4 * kHistWords; i += blockDim.x) (&s_hist[0][0])[i] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // (the trip count is uniform over the workgroup: the histogram adds are
  // made by whole waves)
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < n; b += stride) {
    const int64_t g = b + threadIdx.x;
    const bool valid = g < n;
    uint32_t key = 0u;
    if (valid) {
      const double z = (((double)r0 * (double)means[3 * g] + (double)r1 * (double)means[3 * g + 1]) +
                        (double)r2 * (double)means[3 * g + 2]) + (double)t;
      float zf = (float)z;
      if (zf == 0.0f) zf = 0.0f;
      const uint32_t u = __float_as_uint(zf);
      key = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
      keys[g] = key;
      idx[g] = (uint32_t)g;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) wave_hist_add(s_hist[p], (key >> (8 * p)) & 255u, valid, 8);
  }
  __syncthreads();
  uint32_t *hc = hist_copy(hist);
  for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) {
    const uint32_t c = hist_total(s_hist[i >> 8], i & 255);
    if (c) atomicAdd(&hc[i], c);
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
  job.cnt = w.dcnt;
  job.stride = w.dchunk_stride;
  void *keys[2] = {w.dkeys[0], w.dkeys[1]};
  return sort_passes<uint32_t>(job, 4, 32, (n + kSortChunk - 1) / kSortChunk, keys, w.dvals, s);
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
