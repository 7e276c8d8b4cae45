// Tile binning (Sec. 3.2.1, Fig. 1 stage 3): exclusive scan of per-record tile
// counts, emission of (key, value) pairs with key = global tile << 32 | bits of
// z_start (z_start > 0 after the cull, so the float bits order like the
// values) and value = record index, a stable LSD radix sort over the key bits
// in use, and per-tile [start, end) ranges.  Each record emits in its own slot
// range in row-major tile order and records are ordered by (view, surfel), so
// the sorted order within a tile is (z_start, record): deterministic.
//
// Every kernel reads the data-dependent pair count from device memory and is
// sized by the reserved capacity on the host, so the whole sequence can be
// captured in a HIP graph.
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

// ---------------------------------------------------------------- scan
// Exclusive scan of u32 in three kernels: block sums, scan of the block sums
// (one block), per-block scan plus carry.  Blocks hold 1024 elements.
constexpr int kScanBlock = 1024;

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

__global__ void __launch_bounds__(256) scan_reduce_kernel(const uint32_t* in, long long n, uint32_t* sums) {
  __shared__ uint32_t sh[264];
  long long base = (long long)blockIdx.x * kScanBlock;
  uint32_t s = 0;
  for (int k = 0; k < 4; ++k) {
    long long i = base + k * 256 + threadIdx.x;
    if (i < n) s += in[i];
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

__global__ void __launch_bounds__(256) scan_apply_kernel(const uint32_t* in, uint32_t* out, long long n,
                                                         const uint32_t* sums) {
  __shared__ uint32_t sh[264];
  long long base = (long long)blockIdx.x * kScanBlock;
  // thread t owns 4 consecutive elements
  uint32_t v[4], s = 0;
  for (int k = 0; k < 4; ++k) {
    long long i = base + threadIdx.x * 4 + k;
    v[k] = i < n ? in[i] : 0u;
    s += v[k];
  }
  uint32_t ex = block_exclusive_scan_256(s, sh, nullptr) + sums[blockIdx.x];
  for (int k = 0; k < 4; ++k) {
    long long i = base + threadIdx.x * 4 + k;
    if (i < n) out[i] = ex;
    ex += v[k];
  }
}

long long scan_tmp_size(long long n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, long long n, uint32_t* total,
                           uint32_t* tmp, long long tmp_n, hipStream_t st) {
  long long nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb <= 0 || nb > tmp_n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, st, in, n, tmp);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, st, tmp, nb, total);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(256), 0, st, in, out, n, tmp);
  return hipGetLastError();
}

// ---------------------------------------------------------------- emission
__global__ void __launch_bounds__(256) emit_kernel(const float* __restrict__ recs, const uint32_t* __restrict__ offsets,
                                                   const ViewDev* __restrict__ views, int v0, int tile_w,
                                                   int tile_h, uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals, const uint32_t* n_pairs,
                                                   long long cap, int* status) {
  const ViewDev& v = views[v0 + blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.n_surf) return;
  const long long r = v.rec_off + i;
  const float4 q = reinterpret_cast<const float4*>(recs + r * kRecFloats)[3];
  const int rx = __float_as_int(q.x), ry = __float_as_int(q.y);
  const int il = rx & 0xffff, ih = rx >> 16, jl = ry & 0xffff, jh = ry >> 16;
  if (il > ih || jl > jh) return;
  const int tx0 = il / tile_w, tx1 = ih / tile_w, ty0 = jl / tile_h, ty1 = jh / tile_h;
  const uint32_t zb = (uint32_t)__float_as_int(q.z);
  long long o = offsets[r];
  const long long need = o + (long long)(tx1 - tx0 + 1) * (ty1 - ty0 + 1);
  if (need > cap || need > (long long)*n_pairs) {
    *status = 3;  // SS_ERR_CAPACITY
    return;
  }
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx) {
      const uint64_t tile = (uint64_t)(v.tile_base + ty * v.tiles_x + tx);
      keys[o] = (tile << 32) | zb;
      vals[o] = (uint32_t)r;
      ++o;
    }
}

hipError_t launch_emit_pairs(const float* recs, const uint32_t* offsets, const ViewDev* views,
                             int v0, int v1, int max_surf, int tile_w, int tile_h,
                             uint64_t* keys, uint32_t* vals, const uint32_t* n_pairs,
                             long long cap, int* status, hipStream_t st) {
  if (v1 <= v0 || max_surf <= 0) return hipSuccess;
  dim3 grid((max_surf + 255) / 256, v1 - v0);
  hipLaunchKernelGGL(emit_kernel, grid, dim3(256), 0, st, recs, offsets, views, v0, tile_w, tile_h,
                     keys, vals, n_pairs, cap, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort
// LSD, 8-bit digits.  A block owns kSortItems consecutive pairs; the scatter
// ranks equal digits stably with wave64 ballots (a match-any over the 8 digit
// bits) and per-wave digit counts in LDS.
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortItems = kSortThreads * kSortRounds;

__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(const uint64_t* __restrict__ keys,
                                                                  const uint32_t* n_pairs, int shift,
                                                                  uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const long long n = *n_pairs;
  const long long base = (long long)blockIdx.x * kSortItems;
  for (int k = 0; k < kSortRounds; ++k) {
    long long i = base + k * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(long long)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* n_pairs, int shift, const uint32_t* __restrict__ hist,
    int nblocks) {
  __shared__ uint32_t base_d[256];
  __shared__ uint32_t wc[4][256];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const long long n = *n_pairs;
  const long long base = (long long)blockIdx.x * kSortItems;
  if (base >= n) return;
  base_d[t] = hist[(long long)t * nblocks + blockIdx.x];
  for (int w = 0; w < 4; ++w) wc[w][t] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int k = 0; k < kSortRounds; ++k) {
    const long long i = base + k * kSortThreads + t;
    const bool live = i < n;
    uint64_t key = 0;
    uint32_t val = 0, d = 0;
    if (live) {
      key = kin[i];
      val = vin[i];
      d = (uint32_t)(key >> shift) & 255u;
    }
    uint64_t mask = __ballot(live);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      mask &= bit ? bb : ~bb;
    }
    const int rank = __popcll(mask & lt);
    const int cnt = __popcll(mask);
    const bool leader = live && rank == 0;
    if (leader) wc[wave][d] = (uint32_t)cnt;
    __syncthreads();
    if (live) {
      uint32_t off = base_d[d] + (uint32_t)rank;
      for (int w = 0; w < wave; ++w) off += wc[w][d];
      kout[off] = key;
      vout[off] = val;
    }
    __syncthreads();
    if (leader) {
      atomicAdd(&base_d[d], (uint32_t)cnt);
      wc[wave][d] = 0;
    }
    __syncthreads();
  }
}

hipError_t launch_radix_sort(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp,
                             const uint32_t* n_pairs, long long cap, int key_bits, uint32_t* hist,
                             uint32_t* scan_tmp, long long scan_tmp_n, hipStream_t st,
                             bool* result_in_tmp) {
  const int nblocks = (int)((cap + kSortItems - 1) / kSortItems);
  uint64_t* ka = keys;
  uint32_t* va = vals;
  uint64_t* kb = keys_tmp;
  uint32_t* vb = vals_tmp;
  bool in_tmp = false;
  for (int shift = 0; shift < key_bits; shift += 8) {
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nblocks), dim3(kSortThreads), 0, st, ka, n_pairs,
                       shift, hist, nblocks);
    hipError_t e = launch_scan_u32(hist, hist, (long long)256 * nblocks, nullptr, scan_tmp,
                                   scan_tmp_n, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblocks), dim3(kSortThreads), 0, st, ka, va, kb, vb,
                       n_pairs, shift, hist, nblocks);
    uint64_t* tk = ka; ka = kb; kb = tk;
    uint32_t* tv = va; va = vb; vb = tv;
    in_tmp = !in_tmp;
  }
  *result_in_tmp = in_tmp;
  return hipGetLastError();
}

// ---------------------------------------------------------------- ranges
__global__ void tile_ranges_kernel(const uint64_t* __restrict__ keys, const uint32_t* n_pairs,
                                   long long cap, uint32_t* __restrict__ ranges) {
  const long long n = *n_pairs;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n && i < cap;
       i += (long long)gridDim.x * blockDim.x) {
    const uint32_t tile = (uint32_t)(keys[i] >> 32);
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != tile) ranges[2 * (long long)tile] = (uint32_t)i;
    if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != tile) ranges[2 * (long long)tile + 1] = (uint32_t)(i + 1);
  }
}

hipError_t launch_tile_ranges(const uint64_t* keys, const uint32_t* n_pairs, long long cap,
                              uint32_t* ranges, int tile_begin, int n_tiles, hipStream_t st) {
  hipError_t e = launch_fill_u32(ranges + 2LL * tile_begin, 0u, 2LL * n_tiles, st);
  if (e != hipSuccess) return e;
  long long b = (cap + 255) / 256;
  unsigned nb = (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
  hipLaunchKernelGGL(tile_ranges_kernel, dim3(nb), dim3(256), 0, st, keys, n_pairs, cap, ranges);
  return hipGetLastError();
}

}  // namespace ss
