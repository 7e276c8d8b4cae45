// Tile binning (Sec. 3.2.1, Fig. 1 stage 3).  Order within a tile is by
// (z_start, record index): deterministic, and the order the oracle defines.
// Instead of one sort over (tile, z_start) keys of every pair, the records are
// sorted first and the pairs second, both with 32-bit keys:
//   1. the group's records are radix sorted by the bits of z_start (positive
//      after the cull, so the float bits order like the values; culled
//      records carry 0xffffffff and sort last) with their index as value;
//   2. an exclusive scan of the per-record tile counts, taken in that order,
//      gives each record its slot range;
//   3. each record emits (tile, record) pairs into its slots, tile relative to
//      the group's first tile;
//   4. a stable radix sort over the tile bits in use, then per-tile
//      [start, end) ranges.
// Both sorts are stable and the records enter step 1 in index order, so
// within a tile the result is ordered by (z_start, record index).
//
// Every kernel reads the data-dependent pair count from device memory and is
// sized by the reserved capacity on the host, so the whole sequence can be
// captured in a HIP graph.
#include <type_traits>

#include "common.h"

namespace ss {

// ---------------------------------------------------------------- fills
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_f32_kernel(float* p, float v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
static unsigned fill_blocks(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_blocks(n)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, float v, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32_kernel, dim3(fill_blocks(n)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

// Non-finite entries of p[0..n): a per-lane count, one 64-bit atomic per lane
// that found any (they are rare).
__global__ void count_nonfinite_kernel(const float* __restrict__ p, long long n, unsigned long long* cnt) {
  unsigned c = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    c += isfinite(p[i]) ? 0u : 1u;
  if (c) atomicAdd(cnt, (unsigned long long)c);
}
// NaN into p[0..n) when the latched status is SS_ERR_CAPACITY (3).
__global__ void poison_if_capacity_kernel(float* p, long long n, const int* __restrict__ status) {
  if (*status != 3) return;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = __builtin_nanf("");
}
hipError_t launch_poison_if_capacity(float* p, long long n, const int* status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(poison_if_capacity_kernel, dim3(fill_blocks(n)), dim3(256), 0, st, p, n, status);
  return hipGetLastError();
}
hipError_t launch_count_nonfinite(const float* p, long long n, unsigned long long* cnt, hipStream_t st) {
  if (n <= 0 || !p) return hipSuccess;
  hipLaunchKernelGGL(count_nonfinite_kernel, dim3(fill_blocks(n)), dim3(256), 0, st, p, n, cnt);
  return hipGetLastError();
}

// ---------------------------------------------------------------- deterministic record sums
__global__ void invert_order_kernel(const uint32_t* __restrict__ zidx, long long n, uint32_t* __restrict__ inv) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) inv[zidx[i]] = (uint32_t)i;
}
hipError_t launch_invert_order(const uint32_t* zidx, long long n, uint32_t* inv, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(invert_order_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, zidx, n, inv);
  return hipGetLastError();
}
// One thread per depth-sorted record: its gradient row is the sum, in emission
// order and sub-tile order, of the partials at its pairs' emission slots (slots
// past the pair capacity, after an overflow, are left out).
__global__ void ordered_record_sums_kernel(const uint32_t* __restrict__ zidx, const uint2* __restrict__ zrect,
                                           const uint32_t* __restrict__ offs, long long n, int tile_w, int tile_h,
                                           const float* __restrict__ pgrad, long long pair_base,
                                           long long pair_cap, float* __restrict__ grad) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint2 q = zrect[i];
  const int il = (int)(q.x & 0xffffu), ih = (int)(q.x >> 16), jl = (int)(q.y & 0xffffu), jh = (int)(q.y >> 16);
  float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = s0, s2 = s0, s3 = s0;
  if (il <= ih && jl <= jh) {
    const long long cnt = (long long)(ih / tile_w - il / tile_w + 1) * (jh / tile_h - jl / tile_h + 1);
    const long long o = offs[i], nsub = sub_tiles(tile_w, tile_h);
    const long long k1 = (o + cnt < pair_cap ? o + cnt : pair_cap) * nsub;
    for (long long k = o * nsub; k < k1; ++k) {
      const float4* p = reinterpret_cast<const float4*>(pgrad + (pair_base * nsub + k) * kGradStride);
      const float4 a = p[0], b = p[1], c = p[2], d = p[3];
      s0.x += a.x; s0.y += a.y; s0.z += a.z; s0.w += a.w;
      s1.x += b.x; s1.y += b.y; s1.z += b.z; s1.w += b.w;
      s2.x += c.x; s2.y += c.y; s2.z += c.z; s2.w += c.w;
      s3.x += d.x; s3.y += d.y; s3.z += d.z; s3.w += d.w;
    }
  }
  float4* g = reinterpret_cast<float4*>(grad + (long long)zidx[i] * kGradStride);
  g[0] = s0;
  g[1] = s1;
  g[2] = s2;
  g[3] = s3;
}
hipError_t launch_ordered_record_sums(const uint32_t* zidx, const uint2* zrect, const uint32_t* offs, long long n,
                                      int tile_w, int tile_h, const float* pgrad, long long pair_base,
                                      long long pair_cap, float* grad, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ordered_record_sums_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, zidx, zrect,
                     offs, n, tile_w, tile_h, pgrad, pair_base, pair_cap, grad);
  return hipGetLastError();
}

// ---------------------------------------------------------------- scan
// Exclusive scan of u32 in three kernels: block sums, scan of the block sums
// (one block), per-block scan plus carry.  Blocks of 256 threads hold
// kScanBlock elements.  The scanned sequence is a plain array or the tile
// counts of record rectangles.  Reads are clamped into range rather than
// branched round, so a thread's loads are all in flight at once.
constexpr int kScanPer = 16;
constexpr int kScanBlock = 256 * kScanPer;

struct ScanPlain {
  const uint32_t* in;
  __device__ uint32_t operator()(long long i) const { return in[i]; }
};
// Tiles covered by a record's pixel rectangle (il | ih << 16, jl | jh << 16);
// zero for an empty one (a culled record).
struct ScanRectTiles {
  const uint2* rect;
  int tw, th;
  __device__ uint32_t operator()(long long i) const {
    const uint2 q = rect[i];
    const int il = (int)(q.x & 0xffffu), ih = (int)(q.x >> 16), jl = (int)(q.y & 0xffffu), jh = (int)(q.y >> 16);
    if (il > ih || jl > jh) return 0u;
    return (uint32_t)((ih / tw - il / tw + 1) * (jh / th - jl / th + 1));
  }
};

__device__ inline uint32_t block_exclusive_scan_256(uint32_t v, uint32_t* sh, uint32_t* total) {
  // sh: 256 + 8 entries of LDS
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[256 + wave] = x;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < wave; ++w) base += sh[256 + w];
  uint32_t tot = sh[256] + sh[257] + sh[258] + sh[259];
  __syncthreads();
  if (total) *total = tot;
  return base + x - v;
}

template <class F>
__global__ void __launch_bounds__(256) scan_reduce_kernel(F f, long long n, uint32_t* sums) {
  __shared__ uint32_t sh[264];
  long long base = (long long)blockIdx.x * kScanBlock;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const long long i = base + k * 256 + threadIdx.x;
    const uint32_t x = f(i < n ? i : n - 1);
    s += i < n ? x : 0u;
  }
  uint32_t tot;
  block_exclusive_scan_256(s, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) scan_sums_kernel(uint32_t* sums, long long nb, uint32_t* total) {
  __shared__ uint32_t sh[264];
  uint32_t carry = 0;
  for (long long c = 0; c < nb; c += 256) {
    long long i = c + threadIdx.x;
    uint32_t v = i < nb ? sums[i] : 0u;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan_256(v, sh, &tot);
    if (i < nb) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// In place is fine: a block reads all its elements before writing any.  Loads
// and stores are coalesced; LDS (rows padded against bank conflicts) turns
// them into kScanPer consecutive elements per thread and back.
template <class F>
__global__ void __launch_bounds__(256) scan_apply_kernel(F f, uint32_t* out, long long n, const uint32_t* sums) {
  constexpr int kRow = kScanPer + 1;
  __shared__ uint32_t sh[264];
  __shared__ uint32_t tv[256 * kRow];
  const int t = threadIdx.x;
  const long long base = (long long)blockIdx.x * kScanBlock;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int j = k * 256 + t;
    const long long i = base + j;
    const uint32_t x = f(i < n ? i : n - 1);
    tv[(j / kScanPer) * kRow + j % kScanPer] = i < n ? x : 0u;
  }
  __syncthreads();
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) s += tv[t * kRow + k];
  uint32_t ex = block_exclusive_scan_256(s, sh, nullptr) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const uint32_t x = tv[t * kRow + k];
    tv[t * kRow + k] = ex;
    ex += x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int j = k * 256 + t;
    const long long i = base + j;
    if (i < n) out[i] = tv[(j / kScanPer) * kRow + j % kScanPer];
  }
}

long long scan_tmp_size(long long n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

template <class F>
static hipError_t scan_with(F f, uint32_t* out, long long n, uint32_t* total, uint32_t* tmp, long long tmp_n,
                            hipStream_t st) {
  long long nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb <= 0 || nb > tmp_n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scan_reduce_kernel<F>, dim3((unsigned)nb), dim3(256), 0, st, f, n, tmp);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, st, tmp, nb, total);
  hipLaunchKernelGGL(scan_apply_kernel<F>, dim3((unsigned)nb), dim3(256), 0, st, f, out, n, tmp);
  return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, long long n, uint32_t* total, uint32_t* tmp,
                           long long tmp_n, hipStream_t st) {
  return scan_with(ScanPlain{in}, out, n, total, tmp, tmp_n, st);
}

hipError_t launch_scan_rect_tiles(const uint2* rect, int tile_w, int tile_h, uint32_t* out, long long n,
                                  uint32_t* total, uint32_t* tmp, long long tmp_n, hipStream_t st) {
  return scan_with(ScanRectTiles{rect, tile_w, tile_h}, out, n, total, tmp, tmp_n, st);
}

// ---------------------------------------------------------------- raster work items
// Segments of the tile at position k of the order: one, or ceil(len / seg_len)
// for a list longer than the split threshold.  SPLIT: count only split tiles.
__device__ inline uint32_t seg_count(const uint32_t* ranges, int tile, uint32_t seg_len, uint32_t thr) {
  const uint32_t len = ranges[2 * tile + 1] - ranges[2 * tile];
  return len > thr ? (len + seg_len - 1) / seg_len : 1u;
}
__device__ inline uint32_t split_threshold(const uint32_t* n_pairs, uint32_t seg_len, uint32_t waves_per_tile) {
  const uint32_t t = (uint32_t)(2ull * *n_pairs * waves_per_tile / kResidentWaves);
  return t > seg_len ? t : seg_len;
}
template <bool SPLIT>
struct ScanSegs {
  const uint32_t* ranges;
  const int* order;
  uint32_t seg_len, wpt;
  const uint32_t* n_pairs;
  __device__ uint32_t operator()(long long k) const {
    const uint32_t n = seg_count(ranges, order[k], seg_len, split_threshold(n_pairs, seg_len, wpt));
    return SPLIT ? (n > 1u ? n : 0u) : n;
  }
};

__global__ void seg_items_kernel(const uint32_t* __restrict__ ranges, const int* __restrict__ order, int n_tiles,
                                 uint32_t seg_len, uint32_t wpt, const uint32_t* __restrict__ n_pairs,
                                 const uint32_t* __restrict__ base, const uint32_t* __restrict__ mbase,
                                 int4* __restrict__ items, int4* __restrict__ mitems, long long cap, long long mcap) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_tiles) return;
  const int tile = order[k];
  const int n = (int)seg_count(ranges, tile, seg_len, split_threshold(n_pairs, seg_len, wpt));
  for (int s = 0; s < n; ++s) {
    const long long i = (long long)base[k] + s, m = n > 1 ? (long long)mbase[k] + s : -1;
    const int4 it = make_int4(tile, s, n, (int)m);
    if (i < cap) items[i] = it;
    if (m >= 0 && m < mcap) mitems[m] = it;
  }
}

hipError_t launch_seg_items(const uint32_t* ranges, const int* order, int n_tiles, int seg_len, int tile_pixels,
                            const uint32_t* n_pairs, uint32_t* base, uint32_t* counts, int4* items, int4* mitems,
                            long long items_cap, long long mitems_cap, uint32_t* tmp, long long tmp_n,
                            hipStream_t st) {
  if (n_tiles <= 0 || seg_len <= 0 || tile_pixels < 64) return hipErrorInvalidValue;
  const uint32_t sl = (uint32_t)seg_len, wpt = (uint32_t)(tile_pixels / 64);
  hipError_t e = scan_with(ScanSegs<false>{ranges, order, sl, wpt, n_pairs}, base, n_tiles, counts, tmp, tmp_n, st);
  if (e != hipSuccess) return e;
  e = scan_with(ScanSegs<true>{ranges, order, sl, wpt, n_pairs}, base + n_tiles, n_tiles, counts + 1, tmp, tmp_n,
                st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(seg_items_kernel, dim3((n_tiles + 255) / 256), dim3(256), 0, st, ranges, order, n_tiles, sl,
                     wpt, n_pairs, base, base + n_tiles, items, mitems, items_cap, mitems_cap);
  return hipGetLastError();
}

// ---------------------------------------------------------------- emission
// Position i of the depth-sorted record list (record order[i], pixel rectangle
// rect[i]) emits its pairs into slots offsets[i] on, in row-major order of its
// tile rectangle.  The records of a block fill one contiguous slot range; it is
// staged in LDS in windows of kEmitWindow slots and written out coalesced.
constexpr int kEmitThreads = 256;
constexpr int kEmitWindow = 2048;

__global__ void __launch_bounds__(kEmitThreads) emit_kernel(const uint32_t* __restrict__ order,
                                                            const uint2* __restrict__ rect,
                                                            const uint32_t* __restrict__ offsets,
                                                            const ViewDev* __restrict__ views, int v0, int nv,
                                                            int tile_w, int tile_h, long long n_rec,
                                                            uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                            long long cap, int* status) {
  __shared__ long long roff[kMaxViews];
  __shared__ int tbase[kMaxViews], tilesx[kMaxViews];
  __shared__ uint32_t sk[kEmitWindow], sv[kEmitWindow];
  __shared__ long long span[2];
  const int t = threadIdx.x;
  if (t < nv) {
    const ViewDev& v = views[v0 + t];
    roff[t] = v.rec_off;
    tbase[t] = v.tile_base - views[v0].tile_base;
    tilesx[t] = v.tiles_x;
  }
  const long long i0 = (long long)blockIdx.x * kEmitThreads;
  const long long i1 = i0 + kEmitThreads < n_rec ? i0 + kEmitThreads : n_rec;
  if (t == 0) {
    span[0] = offsets[i0];
    span[1] = 0;
  }
  __syncthreads();
  const long long i = i0 + t;
  uint32_t r = 0u;
  long long o = 0, cnt = 0;
  int tx0 = 0, ty0 = 0, nx = 1, tb = 0, tx = 0;
  if (i < i1) {
    r = order[i];
    o = offsets[i];
    const uint2 q = rect[i];
    const int il = (int)(q.x & 0xffffu), ih = (int)(q.x >> 16), jl = (int)(q.y & 0xffffu), jh = (int)(q.y >> 16);
    if (il <= ih && jl <= jh) {
      int lo = 0, hi = nv - 1;  // the view holding record r: last one with rec_off <= r
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (roff[mid] <= (long long)r) lo = mid;
        else hi = mid - 1;
      }
      tx0 = il / tile_w;
      ty0 = jl / tile_h;
      nx = ih / tile_w - tx0 + 1;
      cnt = (long long)nx * (jh / tile_h - ty0 + 1);
      tb = tbase[lo];
      tx = tilesx[lo];
      if (o + cnt > cap) *status = 3;  // SS_ERR_CAPACITY; every slot below cap is still written
    }
    if (i == i1 - 1) span[1] = o + cnt;
  }
  __syncthreads();
  const long long s0 = span[0], s1 = span[1] < cap ? span[1] : cap;
  for (long long w = s0; w < s1; w += kEmitWindow) {
    const long long we = w + kEmitWindow < s1 ? w + kEmitWindow : s1;
    const long long a = o > w ? o : w, e = o + cnt < we ? o + cnt : we;
    if (a < e) {
      int j = (int)(a - o);
      int dy = j / nx, dx = j - dy * nx;
      for (long long s = a; s < e; ++s) {
        sk[s - w] = (uint32_t)(tb + (ty0 + dy) * tx + tx0 + dx);
        sv[s - w] = r;
        if (++dx == nx) {
          dx = 0;
          ++dy;
        }
      }
    }
    __syncthreads();
    for (long long s = w + t; s < we; s += kEmitThreads) {
      keys[s] = sk[s - w];
      vals[s] = sv[s - w];
    }
    __syncthreads();
  }
}

hipError_t launch_emit_pairs(const uint32_t* order, const uint2* rect, const uint32_t* offsets,
                             const ViewDev* views, int v0, int v1, long long n_rec, int tile_w, int tile_h,
                             uint32_t* keys, uint32_t* vals, long long cap, int* status, hipStream_t st) {
  if (v1 <= v0 || n_rec <= 0) return hipSuccess;
  if (v1 - v0 > kMaxViews) return hipErrorInvalidValue;
  const long long nb = (n_rec + kEmitThreads - 1) / kEmitThreads;
  hipLaunchKernelGGL(emit_kernel, dim3((unsigned)nb), dim3(kEmitThreads), 0, st, order, rect, offsets, views, v0,
                     v1 - v0, tile_w, tile_h, n_rec, keys, vals, cap, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort
// Stable LSD radix sort of 32-bit keys carrying 32-bit values, 8-bit digits
// (the first may have 9, so that 17 key bits take two passes), reduce-then-scan.  The input is cut into chunks of kRadixItems pairs; each
// workgroup owns a contiguous run of chunks, each of its waves a contiguous
// 1/8 of a chunk, so workgroup, chunk and wave order are the input order.
// Per pass: the histogram kernel writes each workgroup's digit counts
// digit-major (hist[digit * groups + group]), one exclusive scan of that array
// gives every workgroup the global start of each digit's run, and the scatter
// kernel walks its chunks in order: it ranks each pair stably inside the chunk
// (wave64 match-any over the digit bits, per-wave running digit counts),
// stages the chunk in LDS in digit order and writes every digit's run of the
// chunk to consecutive addresses after the runs of the chunks before it.
constexpr int kRadixThreads = 512;
constexpr int kRadixWaves = kRadixThreads / 64;
constexpr int kRadixRounds = 16;
constexpr int kRadixPerWave = 64 * kRadixRounds;
constexpr int kRadixItems = kRadixThreads * kRadixRounds;
constexpr int kRadixMaxGroups = 1 << 20;

struct RadixGrid {
  int groups, chunks_per_group;
};
static RadixGrid radix_grid(long long cap) {
  const long long chunks = (cap + kRadixItems - 1) / kRadixItems;
  RadixGrid g;
  g.chunks_per_group = (int)((chunks + kRadixMaxGroups - 1) / kRadixMaxGroups);
  if (g.chunks_per_group < 1) g.chunks_per_group = 1;
  g.groups = (int)((chunks + g.chunks_per_group - 1) / g.chunks_per_group);
  if (g.groups < 1) g.groups = 1;
  return g;
}
long long radix_hist_size(long long cap) { return 512LL * radix_grid(cap).groups; }  // up to 9-bit digits

__device__ inline long long radix_count(const uint32_t* n_dev, long long n_fixed, long long cap) {
  const long long n = n_fixed >= 0 ? n_fixed : (long long)*n_dev;
  return n < cap ? n : cap;
}

// Lanes of the wave holding the same BITS-bit digit as this one, among live lanes.
template <int BITS>
__device__ inline uint64_t match_digit(uint32_t d, bool live) {
  uint64_t m = __ballot(live);
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ inline uint64_t lanes_below() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull) >> (64 - lane);
}

template <int BITS>
__global__ void __launch_bounds__(kRadixThreads) radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                                   const uint32_t* n_dev, long long n_fixed,
                                                                   long long cap, int shift, int cpg,
                                                                   uint32_t* __restrict__ hist) {
  // sub-histograms per wave (by lane: 4 for 8-bit digits, 2 for 9-bit ones)
  // cut same-address conflicts of the LDS atomics on skewed digits; rows padded
  // by one entry to put them in other banks
  constexpr int NB = 1 << BITS, kSub = BITS == 8 ? 4 : 2, kRow = NB + 1;
  static_assert(NB <= kRadixThreads, "one thread per digit");
  __shared__ uint32_t wh[kRadixWaves * kSub * kRow];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  uint32_t* my = wh + (wave * kSub + (lane & (kSub - 1))) * kRow;
  for (int i = t; i < kRadixWaves * kSub * kRow; i += kRadixThreads) wh[i] = 0u;
  __syncthreads();
  const long long n = radix_count(n_dev, n_fixed, cap);
  for (int c = 0; c < cpg; ++c) {
    const long long b0 = ((long long)blockIdx.x * cpg + c) * kRadixItems;
    if (b0 >= n) break;
    const long long base = b0 + (long long)wave * kRadixPerWave + lane;
    // loads clamped into range (n > b0 >= 0), not branched round, so all are in flight at once
    uint32_t d[kRadixRounds];
#pragma unroll
    for (int k = 0; k < kRadixRounds; ++k) {
      const long long i = base + 64 * k;
      d[k] = (keys[i < n ? i : n - 1] >> shift) & (NB - 1u);
    }
#pragma unroll
    for (int k = 0; k < kRadixRounds; ++k)
      if (base + 64 * k < n) atomicAdd(&my[d[k]], 1u);
  }
  __syncthreads();
  if (t < NB) {
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < kRadixWaves * kSub; ++w) s += wh[w * kRow + t];
    hist[(long long)t * gridDim.x + blockIdx.x] = s;
  }
}

// IOTA: the input values are val0 + (input position), vin is not read.
// GATHER: also writes gout[dst] = gsrc[value] (the last pass of a sort whose
// values index gsrc), or gskip_val without reading gsrc where the key is
// gskip_key (entries whose gathered value is known: culled records).
template <bool IOTA, bool GATHER, int BITS>
__global__ void __launch_bounds__(kRadixThreads) radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t val0,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const uint2* __restrict__ gsrc,
    uint2* __restrict__ gout, uint32_t gskip_key, uint2 gskip_val, const uint32_t* n_dev, long long n_fixed,
    long long cap, int shift, int cpg, const uint32_t* __restrict__ hist) {
  constexpr int NB = 1 << BITS;
  // per-wave digit counts, then chunk-local run starts (both below kRadixItems,
  // so 16 bits hold them for 9-bit digits and two blocks still fit a CU's LDS)
  using Cnt = typename std::conditional<BITS == 8, uint32_t, uint16_t>::type;
  static_assert(NB <= kRadixThreads && kRadixItems <= 65536, "one thread per digit, 16-bit positions");
  __shared__ Cnt woff[kRadixWaves][NB];
  __shared__ uint32_t loc[NB];                 // chunk-local start of each digit
  __shared__ uint32_t run[NB];                 // global start of each digit's run of this chunk
  __shared__ uint32_t wsum[NB / 64];
  __shared__ uint32_t sk[kRadixItems];
  __shared__ uint32_t sv[kRadixItems];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const long long n = radix_count(n_dev, n_fixed, cap);
  if (t < NB) run[t] = hist[(long long)t * gridDim.x + blockIdx.x];
  const uint64_t lt = lanes_below();
  for (int c = 0; c < cpg; ++c) {
    const long long b0 = ((long long)blockIdx.x * cpg + c) * kRadixItems;
    if (b0 >= n) break;
    for (int i = t; i < kRadixWaves * NB; i += kRadixThreads) (&woff[0][0])[i] = 0u;
    const long long base = b0 + (long long)wave * kRadixPerWave + lane;
    // loads clamped into range (n > b0 >= 0), not branched round, so all are in flight at once
    uint32_t key[kRadixRounds], val[kRadixRounds];
#pragma unroll
    for (int k = 0; k < kRadixRounds; ++k) {
      const long long i = base + 64 * k;
      const long long ic = i < n ? i : n - 1;
      key[k] = kin[ic];
      val[k] = IOTA ? val0 + (uint32_t)i : vin[ic];
    }
    __syncthreads();
    // stable rank of each pair among the wave's pairs of its digit
    uint32_t pre[kRadixRounds];
#pragma unroll
    for (int k = 0; k < kRadixRounds; ++k) {
      const bool live = base + 64 * k < n;
      const uint32_t d = (key[k] >> shift) & (NB - 1u);
      const uint64_t m = match_digit<BITS>(d, live);
      const uint32_t r = (uint32_t)__popcll(m & lt);
      const uint32_t cw = woff[wave][d];
      pre[k] = cw + r;
      __builtin_amdgcn_wave_barrier();
      if (live && r == 0) woff[wave][d] = (Cnt)(cw + (uint32_t)__popcll(m));
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // digit totals -> exclusive scan over digits -> per-wave run starts
    uint32_t tot = 0, incl = 0;
    if (t < NB) {
#pragma unroll
      for (int w = 0; w < kRadixWaves; ++w) {
        const uint32_t x = woff[w][t];
        woff[w][t] = (Cnt)tot;
        tot += x;
      }
      incl = tot;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      if (lane == 63) wsum[wave] = incl;
    }
    __syncthreads();
    if (t < NB) {
      uint32_t ex = incl - tot;
      for (int w = 0; w < wave; ++w) ex += wsum[w];
      loc[t] = ex;
#pragma unroll
      for (int w = 0; w < kRadixWaves; ++w) woff[w][t] = (Cnt)(woff[w][t] + ex);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRadixRounds; ++k) {
      if (base + 64 * k < n) {
        const uint32_t p = woff[wave][(key[k] >> shift) & (NB - 1u)] + pre[k];
        sk[p] = key[k];
        sv[p] = val[k];
      }
    }
    __syncthreads();
    const int cnt = (int)(n - b0 < kRadixItems ? n - b0 : kRadixItems);
#pragma unroll 4
    for (int p = t; p < cnt; p += kRadixThreads) {
      const uint32_t k = sk[p];
      const uint32_t d = (k >> shift) & (NB - 1u);
      const uint32_t dst = run[d] + ((uint32_t)p - loc[d]);
      const uint32_t v = sv[p];
      kout[dst] = k;
      vout[dst] = v;
      if (GATHER) gout[dst] = k == gskip_key ? gskip_val : gsrc[v];
    }
    __syncthreads();
    if (t < NB) run[t] += tot;
  }
}

hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                             bool iota, uint32_t val0, const uint2* gsrc, uint2* gout, uint32_t gskip_key,
                             uint2 gskip_val, const uint32_t* n_dev, long long n_fixed, long long cap, int passes,
                             int first_bits, uint32_t* hist, long long hist_n, uint32_t* scan_tmp,
                             long long scan_tmp_n, hipStream_t st) {
  if (passes <= 0 || cap <= 0) return hipSuccess;
  if (first_bits != 8 && first_bits != 9) return hipErrorInvalidValue;
  const RadixGrid rg = radix_grid(cap);
  if ((1LL << first_bits) * rg.groups > hist_n) return hipErrorInvalidValue;
  uint32_t *ka = keys, *va = vals, *kb = keys_tmp, *vb = vals_tmp;
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int bits = p == 0 ? first_bits : 8;
    if (bits == 9)
      hipLaunchKernelGGL(radix_hist_kernel<9>, dim3(rg.groups), dim3(kRadixThreads), 0, st, ka, n_dev, n_fixed,
                         cap, shift, rg.chunks_per_group, hist);
    else
      hipLaunchKernelGGL(radix_hist_kernel<8>, dim3(rg.groups), dim3(kRadixThreads), 0, st, ka, n_dev, n_fixed,
                         cap, shift, rg.chunks_per_group, hist);
    hipError_t e = launch_scan_u32(hist, hist, (1LL << bits) * rg.groups, nullptr, scan_tmp, scan_tmp_n, st);
    if (e != hipSuccess) return e;
    const bool io = iota && p == 0, ga = gsrc && p == passes - 1;
#define SS_SCATTER(I, G, B)                                                                                    \
  hipLaunchKernelGGL((radix_scatter_kernel<I, G, B>), dim3(rg.groups), dim3(kRadixThreads), 0, st, ka, va, val0, \
                     kb, vb, gsrc, gout, gskip_key, gskip_val, n_dev, n_fixed, cap, shift, rg.chunks_per_group, hist)
    if (bits == 9) {
      // (a 9-bit digit only ever leads a pair sort: no values by position, no gather)
      if (io || ga) return hipErrorInvalidValue;
      SS_SCATTER(false, false, 9);
    } else if (io && ga) SS_SCATTER(true, true, 8);
    else if (io) SS_SCATTER(true, false, 8);
    else if (ga) SS_SCATTER(false, true, 8);
    else SS_SCATTER(false, false, 8);
#undef SS_SCATTER
    shift += bits;
    uint32_t* tk = ka; ka = kb; kb = tk;
    uint32_t* tv = va; va = vb; vb = tv;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- ranges
// keys: sorted tile indices relative to tile_begin.  A block stages
// kRangeItems keys and one neighbour on each side in LDS (coalesced loads,
// clamped into range) and marks where the tile changes.
constexpr int kRangeItems = 2048;

__global__ void __launch_bounds__(256) tile_ranges_kernel(const uint32_t* __restrict__ keys, const uint32_t* n_pairs,
                                                          long long cap, int tile_begin,
                                                          uint32_t* __restrict__ ranges) {
  __shared__ uint32_t sk[kRangeItems + 2];
  const long long n = (long long)*n_pairs < cap ? (long long)*n_pairs : cap;
  const long long b0 = (long long)blockIdx.x * kRangeItems;
  if (b0 >= n) return;
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kRangeItems / 256; ++k) {
    const long long i = b0 + k * 256 + t;
    sk[1 + k * 256 + t] = keys[i < n ? i : n - 1];
  }
  if (t == 0) sk[0] = keys[b0 > 0 ? b0 - 1 : 0];
  if (t == 1) sk[kRangeItems + 1] = keys[b0 + kRangeItems < n ? b0 + kRangeItems : n - 1];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRangeItems / 256; ++k) {
    const int j = k * 256 + t;
    const long long i = b0 + j;
    if (i < n) {
      const uint32_t key = sk[1 + j];
      const long long g = (long long)tile_begin + key;
      if (i == 0 || sk[j] != key) ranges[2 * g] = (uint32_t)i;
      if (i == n - 1 || sk[2 + j] != key) ranges[2 * g + 1] = (uint32_t)(i + 1);
    }
  }
}

hipError_t launch_tile_ranges(const uint32_t* keys, const uint32_t* n_pairs, long long cap,
                              uint32_t* ranges, int tile_begin, int n_tiles, hipStream_t st) {
  hipError_t e = launch_fill_u32(ranges + 2LL * tile_begin, 0u, 2LL * n_tiles, st);
  if (e != hipSuccess) return e;
  const long long b = (cap + kRangeItems - 1) / kRangeItems;
  if (b <= 0) return hipSuccess;
  hipLaunchKernelGGL(tile_ranges_kernel, dim3((unsigned)b), dim3(256), 0, st, keys, n_pairs, cap, tile_begin, ranges);
  return hipGetLastError();
}

}  // namespace ss
