// Tile rasterizer, forward and backward (Alg. 1, eq:shepard, eq:alpha,
// eq:compositing, App. A.1).
//
// A block owns one tile of TW x TH pixels; each wave64 owns an 8 x 8 sub-tile,
// one pixel per lane.  The tile's sorted records are staged through LDS in
// batches (one 64-byte record per surfel, coalesced gathers by the whole
// block); every wave first tests the record's pixel rectangle against its own
// sub-tile (wave-uniform skip), then each lane evaluates the MIP-filtered
// weight and runs the interval-merging grouping of Alg. 1.
//
// Forward: per pixel it writes the image, alpha, the layer count and each
// layer's (W_k, C_k) (unnormalised), at most K_max of them.
// Backward: instead of a replay pass it reads those per-layer totals back
// (per pixel, never per fragment), rebuilds T_k, alpha_k, C_hat_k and the
// suffix sums, and re-walks the tile front to back with the identical
// per-fragment evaluation and grouping decisions.  Per fragment it forms
// dL/dw and dL/dc, maps them to the record's 11 parameters, reduces them over
// the wave with cross-lane shuffles and issues one atomic add per value per
// wave.
#include "common.h"

namespace ss {

template <int TW, int TH>
__device__ __forceinline__ void pixel_of_thread(int t, int tile_x, int tile_y, int& lx, int& ly,
                                                int& sx0, int& sy0) {
  const int lane = t & 63, wave = t >> 6;
  constexpr int WX = TW / 8;
  const int wx = wave % WX, wy = wave / WX;
  lx = wx * 8 + (lane & 7);
  ly = wy * 8 + (lane >> 3);
  sx0 = tile_x * TW + wx * 8;
  sy0 = tile_y * TH + wy * 8;
}

// Does the record's pixel rectangle meet the 8 x 8 sub-tile at (sx0, sy0)?
__device__ __forceinline__ bool rect_meets(const float4 q, int sx0, int sy0) {
  const int rx = __float_as_int(q.x), ry = __float_as_int(q.y);
  const int il = rx & 0xffff, ih = rx >> 16, jl = ry & 0xffff, jh = ry >> 16;
  return !(ih < sx0 || il > sx0 + 7 || jh < sy0 || jl > sy0 + 7);
}

__device__ __forceinline__ void load_batch(float4* lds, const uint32_t* __restrict__ vals,
                                           const float* __restrict__ recs, uint32_t b0, int cnt,
                                           int nthreads) {
  // 4 threads per record, one float4 each
  for (int j = threadIdx.x; j < cnt * 4; j += nthreads) {
    const uint32_t id = vals[b0 + (j >> 2)];
    lds[j] = reinterpret_cast<const float4*>(recs + (size_t)id * kRecFloats)[j & 3];
  }
}

// Wave-level compaction of a chunk of up to 64 staged records: lane j tests
// record c0 + j against the wave's sub-tile; the ballot is the (wave-uniform)
// set of records this wave visits, in list order.
__device__ __forceinline__ uint64_t chunk_mask(const float4* lds, int c0, int cnt, int lane, int sx0,
                                               int sy0) {
  const int j = c0 + lane;
  bool ov = false;
  if (j < cnt) ov = rect_meets(lds[4 * j + 3], sx0, sy0);
  return __ballot(ov);
}

__device__ __forceinline__ int next_item(int* queue, int persistent, int& s_item, int iter) {
  if (!persistent) return iter == 0 ? (int)blockIdx.x : -1;
  if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
  __syncthreads();
  int it = s_item;
  __syncthreads();
  return it;
}

// ---------------------------------------------------------------- forward
template <int TW, int TH>
__global__ void __launch_bounds__(TW* TH) raster_forward_kernel(
    const ViewDev* __restrict__ views, int n_views, int tile_begin, int n_items,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const float* __restrict__ recs, Params prm, int B, float* __restrict__ image,
    float* __restrict__ alpha, uint8_t* __restrict__ nl_out, uint8_t* __restrict__ nl_int,
    float4* __restrict__ stats, int* queue, const int* __restrict__ order, int persistent) {
  extern __shared__ float4 lds[];
  __shared__ int s_item;
  constexpr int NT = TW * TH;
  const int t = threadIdx.x, lane = t & 63;
  const float r2 = prm.r2, kappa = prm.kappa;
  const int kmax = prm.k_max;
  for (int iter = 0;; ++iter) {
    const int item = next_item(queue, persistent, s_item, iter);
    if (item < 0 || item >= n_items) break;
    const int tile = order ? order[item] : tile_begin + item;
    const ViewDev& v = views[view_of_tile(views, n_views, tile)];
    const int lt = tile - v.tile_base;
    const int tx = lt % v.tiles_x, ty = lt / v.tiles_x;
    int lx, ly, sx0, sy0;
    pixel_of_thread<TW, TH>(t, tx, ty, lx, ly, sx0, sy0);
    const int px = tx * TW + lx, py = ty * TH + ly;
    const bool inside = px < v.W && py < v.H;
    const long long pix = v.pix_off + (long long)py * v.W + px;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

    float C0 = 0.f, C1 = 0.f, C2 = 0.f, Wg = 0.f, zmax = 0.f;
    float O0 = 0.f, O1 = 0.f, O2 = 0.f, T = 1.f;
    int K = 0;
    bool done = !inside;
    for (uint32_t b0 = start; b0 < end; b0 += (uint32_t)B) {
      if (__syncthreads_and(done)) break;
      const int cnt = (int)min((uint32_t)B, end - b0);
      load_batch(lds, vals, recs, b0, cnt, NT);
      __syncthreads();
      for (int c0 = 0; c0 < cnt; c0 += 64) {
        if (__ballot(!done) == 0ull) break;
        uint64_t m = chunk_mask(lds, c0, cnt, lane, sx0, sy0);
        while (m) {
          const int j = c0 + __builtin_ctzll(m);
          m &= m - 1;
          const float* rec = reinterpret_cast<const float*>(lds + 4 * j);
          FragEval f;
          frag_eval(rec, px, py, r2, f);
          if (!f.cov || done) continue;
          if (Wg > 0.f && rec[R_ZS] > zmax) {
            // gap: finalise the layer (Shepard-normalised colour, coverage opacity)
            const float a = -expm1f(-kappa * Wg), e = __expf(-kappa * Wg);
            const float s = T * a / Wg;
            O0 += s * C0; O1 += s * C1; O2 += s * C2;
            stats[pix * kMaxLayers + K] = make_float4(Wg, C0, C1, C2);
            T *= e;
            ++K;
            C0 = C1 = C2 = 0.f;
            Wg = 0.f;
            zmax = 0.f;
            if (K >= kmax) { done = true; continue; }
          }
          zmax = fmaxf(zmax, rec[R_ZE]);
          C0 += f.w * rec[R_CR];
          C1 += f.w * rec[R_CG];
          C2 += f.w * rec[R_CB];
          Wg += f.w;
        }
      }
      __syncthreads();
    }
    if (inside) {
      if (!done && Wg > 0.f) {
        const float a = -expm1f(-kappa * Wg), e = __expf(-kappa * Wg);
        const float s = T * a / Wg;
        O0 += s * C0; O1 += s * C1; O2 += s * C2;
        stats[pix * kMaxLayers + K] = make_float4(Wg, C0, C1, C2);
        T *= e;
        ++K;
      }
      image[3 * pix + 0] = O0 + T * v.bg[0];
      image[3 * pix + 1] = O1 + T * v.bg[1];
      image[3 * pix + 2] = O2 + T * v.bg[2];
      alpha[pix] = 1.f - T;
      nl_int[pix] = (uint8_t)K;
      if (nl_out) nl_out[pix] = (uint8_t)K;
    }
  }
}

// ---------------------------------------------------------------- backward
// Sum of x over the 16 lanes of each row, left in every lane of the row
// (quad xor 1, quad xor 2, half-row mirror, row mirror).
__device__ __forceinline__ float row_sum16(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, false));
  return x;
}

// Reduces 12 per-lane values over the wave with a transposed butterfly:
// permlane32_swap pairs (g_i, g_{i+6}) so lanes 0-31 carry value i and lanes
// 32-63 value i+6; permlane16_swap pairs (s_i, s_{i+3}) so row r carries value
// i + 3r; a row sum finishes.  Lane 16r + k (k < 3) returns the total of value
// 3r + k in *vidx, other lanes -1.  Needs all 64 lanes active.
__device__ __forceinline__ float wave_reduce12(const float g[12], int lane, int* vidx) {
  float s[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(g[i]), __float_as_uint(g[i + 6]),
                                                    false, false);
    s[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  float t3[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(s[i]), __float_as_uint(s[i + 3]),
                                                    false, false);
    t3[i] = row_sum16(__uint_as_float(r[0]) + __uint_as_float(r[1]));
  }
  const int row = lane >> 4, k = lane & 15;
  *vidx = k < 3 ? 3 * row + k : -1;
  return k == 0 ? t3[0] : (k == 1 ? t3[1] : t3[2]);
}

struct LayerCoef {
  float W, e, a, Ch0, Ch1, Ch2, dW, coef, GC;
};

__device__ __forceinline__ void layer_coef(const float4 st, float Tk, float kappa, const float G[3],
                                           float ga, float Tfin, const float Cf[3], const float pre[3],
                                           LayerCoef& L) {
  L.W = st.x;
  L.a = -expm1f(-kappa * st.x);
  L.e = __expf(-kappa * st.x);
  const float iW = 1.f / st.x;
  L.Ch0 = st.y * iW; L.Ch1 = st.z * iW; L.Ch2 = st.w * iW;
  const float ta = Tk * L.a;
  // suffix S_k = sum_{j>k} T_j a_j C_j + T_{K+1} bg = C_final - prefix - T_k a_k C_k
  const float S0 = Cf[0] - pre[0] - ta * L.Ch0;
  const float S1 = Cf[1] - pre[1] - ta * L.Ch1;
  const float S2 = Cf[2] - pre[2] - ta * L.Ch2;
  const float Tk1 = Tk * L.e;
  L.dW = kappa * (G[0] * (Tk1 * L.Ch0 - S0) + G[1] * (Tk1 * L.Ch1 - S1) + G[2] * (Tk1 * L.Ch2 - S2) +
                  ga * Tfin);
  L.coef = ta * iW;
  L.GC = G[0] * L.Ch0 + G[1] * L.Ch1 + G[2] * L.Ch2;
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW* TH) raster_backward_kernel(
    const ViewDev* __restrict__ views, int n_views, int tile_begin, int n_items,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const float* __restrict__ recs, Params prm, int B, const float* __restrict__ d_image,
    const float* __restrict__ d_alpha, const uint8_t* __restrict__ nl_int,
    const float4* __restrict__ stats, float* __restrict__ grad, long long R, int* queue,
    const int* __restrict__ order, int persistent) {
  extern __shared__ float4 lds[];
  __shared__ int s_item;
  constexpr int NT = TW * TH;
  const int t = threadIdx.x, lane = t & 63;
  const float r2 = prm.r2, kappa = prm.kappa;
  const int kmax = prm.k_max;
  for (int iter = 0;; ++iter) {
    const int item = next_item(queue, persistent, s_item, iter);
    if (item < 0 || item >= n_items) break;
    const int tile = order ? order[item] : tile_begin + item;
    const ViewDev& v = views[view_of_tile(views, n_views, tile)];
    const int lt = tile - v.tile_base;
    const int tx = lt % v.tiles_x, ty = lt / v.tiles_x;
    int lx, ly, sx0, sy0;
    pixel_of_thread<TW, TH>(t, tx, ty, lx, ly, sx0, sy0);
    const int px = tx * TW + lx, py = ty * TH + ly;
    const bool inside = px < v.W && py < v.H;
    const long long pix = v.pix_off + (long long)py * v.W + px;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

    float G[3] = {0.f, 0.f, 0.f}, ga = 0.f;
    int nl = 0;
    float Cf[3] = {0.f, 0.f, 0.f}, pre[3] = {0.f, 0.f, 0.f};
    float Tfin = 1.f, Tk = 1.f;
    LayerCoef L;
    L.W = 1.f; L.e = 1.f; L.a = 0.f; L.Ch0 = L.Ch1 = L.Ch2 = 0.f; L.dW = 0.f; L.coef = 0.f; L.GC = 0.f;
    bool done = true;
    if (inside) {
      G[0] = d_image[3 * pix]; G[1] = d_image[3 * pix + 1]; G[2] = d_image[3 * pix + 2];
      ga = d_alpha ? d_alpha[pix] : 0.f;
      nl = nl_int[pix];
      float T = 1.f;
      for (int k = 0; k < nl; ++k) {
        const float4 st = stats[pix * kMaxLayers + k];
        const float a = -expm1f(-kappa * st.x), e = __expf(-kappa * st.x);
        const float s = T * a / st.x;
        Cf[0] += s * st.y; Cf[1] += s * st.z; Cf[2] += s * st.w;
        T *= e;
      }
      Tfin = T;
      Cf[0] += T * v.bg[0]; Cf[1] += T * v.bg[1]; Cf[2] += T * v.bg[2];
      if (nl > 0) {
        layer_coef(stats[pix * kMaxLayers], 1.f, kappa, G, ga, Tfin, Cf, pre, L);
        done = false;
      }
    }
    int k = 0;
    float Wg = 0.f, zmax = 0.f;
    for (uint32_t b0 = start; b0 < end; b0 += (uint32_t)B) {
      if (__syncthreads_and(done)) break;
      const int cnt = (int)min((uint32_t)B, end - b0);
      load_batch(lds, vals, recs, b0, cnt, NT);
      __syncthreads();
      for (int c0 = 0; c0 < cnt; c0 += 64) {
        if (__ballot(!done) == 0ull) break;
        uint64_t m = chunk_mask(lds, c0, cnt, lane, sx0, sy0);
        while (m) {
          const int j = c0 + __builtin_ctzll(m);
          m &= m - 1;
          const float* rec = reinterpret_cast<const float*>(lds + 4 * j);
          FragEval f;
          frag_eval(rec, px, py, r2, f);
          bool contrib = false;
          float gw = 0.f, gcs = 0.f;
          if (f.cov && !done) {
            bool live = true;
            if (Wg > 0.f && rec[R_ZS] > zmax) {
              // next layer: the forward flushed layer k here
              pre[0] += Tk * L.a * L.Ch0; pre[1] += Tk * L.a * L.Ch1; pre[2] += Tk * L.a * L.Ch2;
              Tk *= L.e;
              ++k;
              if (k >= kmax || k >= nl) {
                done = true;
                live = false;
              } else {
                layer_coef(stats[pix * kMaxLayers + k], Tk, kappa, G, ga, Tfin, Cf, pre, L);
                Wg = 0.f;
                zmax = 0.f;
              }
            }
            if (live) {
              zmax = fmaxf(zmax, rec[R_ZE]);
              Wg += f.w;
              const float Gc = G[0] * rec[R_CR] + G[1] * rec[R_CG] + G[2] * rec[R_CB];
              gw = L.dW + L.coef * (Gc - L.GC);
              gcs = f.w * L.coef;
              contrib = true;
            }
          }
          if (__ballot(contrib) == 0ull) continue;
          // d(rho^2)/d(record) for q = d^T Q d / s^2, s = 1 + a3 dx + b3 dy
          const float is = __builtin_amdgcn_rcpf(f.s), is2 = is * is;
          const float gq = -0.5f * f.w * gw;
          const float dx = f.dx, dy = f.dy, q = f.q;
          const float qxx = rec[R_QXX], qxy2 = rec[R_QXY2], qyy = rec[R_QYY];
          float g[12];
          g[G_X0] = -gq * ((2.f * qxx * dx + qxy2 * dy) * is2 - 2.f * q * rec[R_A3] * is);
          g[G_Y0] = -gq * ((qxy2 * dx + 2.f * qyy * dy) * is2 - 2.f * q * rec[R_B3] * is);
          g[G_QXX] = gq * dx * dx * is2;
          g[G_QXY2] = gq * dx * dy * is2;
          g[G_QYY] = gq * dy * dy * is2;
          g[G_A3] = -2.f * gq * q * dx * is;
          g[G_B3] = -2.f * gq * q * dy * is;
          g[G_NF] = gw * f.w * __builtin_amdgcn_rcpf(rec[R_NF]);
          g[G_CR] = gcs * G[0];
          g[G_CG] = gcs * G[1];
          g[G_CB] = gcs * G[2];
          g[11] = 0.f;
#pragma unroll
          for (int q2 = 0; q2 < 11; ++q2) g[q2] = contrib ? g[q2] : 0.f;
          int vidx;
          const float tot = wave_reduce12(g, lane, &vidx);
          if (vidx >= 0 && vidx < kNGrad && tot != 0.f) {
            const uint32_t id = __float_as_uint(rec[R_ID]);
            atomicAdd(grad + (long long)vidx * R + id, tot);
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- launchers
template <int TW, int TH>
static hipError_t fwd_t(dim3 grid, size_t lds, hipStream_t st, const ViewDev* views, int nv, int tb,
                        int ni, const uint32_t* ranges, const uint32_t* vals, const float* recs,
                        const Params& prm, int B, float* image, float* alpha, uint8_t* nlo,
                        uint8_t* nli, float4* stats, int* queue, const int* order, int pers) {
  hipLaunchKernelGGL((raster_forward_kernel<TW, TH>), grid, dim3(TW * TH), lds, st, views, nv, tb, ni,
                     ranges, vals, recs, prm, B, image, alpha, nlo, nli, stats, queue, order, pers);
  return hipGetLastError();
}
template <int TW, int TH>
static hipError_t bwd_t(dim3 grid, size_t lds, hipStream_t st, const ViewDev* views, int nv, int tb,
                        int ni, const uint32_t* ranges, const uint32_t* vals, const float* recs,
                        const Params& prm, int B, const float* di, const float* da,
                        const uint8_t* nli, const float4* stats, float* grad, long long R, int* queue,
                        const int* order, int pers) {
  hipLaunchKernelGGL((raster_backward_kernel<TW, TH>), grid, dim3(TW * TH), lds, st, views, nv, tb, ni,
                     ranges, vals, recs, prm, B, di, da, nli, stats, grad, R, queue, order, pers);
  return hipGetLastError();
}

static unsigned persistent_grid(int n_items, int threads) {
  // 256 CUs; enough resident blocks to cover the chip several times over
  int per_cu = threads <= 64 ? 16 : (threads <= 128 ? 12 : (threads <= 256 ? 8 : 4));
  long long g = 256LL * per_cu;
  return (unsigned)(g < n_items ? g : (n_items > 0 ? n_items : 1));
}

hipError_t launch_raster_forward(const ViewDev* views, int n_views, int tile_begin, int tile_end,
                                 const uint32_t* ranges, const uint32_t* sorted_vals,
                                 const float* recs, const Params& prm, int lds_batch,
                                 float* image, float* alpha, uint8_t* n_layers_out,
                                 uint8_t* n_layers, float4* layer_stats, int* queue,
                                 const int* order, int persistent, hipStream_t st) {
  const int n_items = tile_end - tile_begin;
  if (n_items <= 0) return hipSuccess;
  const int threads = prm.tile_w * prm.tile_h;
  dim3 grid(persistent ? persistent_grid(n_items, threads) : (unsigned)n_items);
  const size_t lds = (size_t)lds_batch * kRecFloats * sizeof(float);
#define SS_FWD(TW, TH) fwd_t<TW, TH>(grid, lds, st, views, n_views, tile_begin, n_items, ranges, \
                                     sorted_vals, recs, prm, lds_batch, image, alpha,            \
                                     n_layers_out, n_layers, layer_stats, queue, order, persistent)
  switch (prm.tile_w * 100 + prm.tile_h) {
    case 808: return SS_FWD(8, 8);
    case 1608: return SS_FWD(16, 8);
    case 1616: return SS_FWD(16, 16);
    case 3208: return SS_FWD(32, 8);
    case 3216: return SS_FWD(32, 16);
    default: return hipErrorInvalidValue;
  }
#undef SS_FWD
}

hipError_t launch_raster_backward(const ViewDev* views, int n_views, int tile_begin, int tile_end,
                                  const uint32_t* ranges, const uint32_t* sorted_vals,
                                  const float* recs, const Params& prm, int lds_batch,
                                  const float* d_image, const float* d_alpha,
                                  const uint8_t* n_layers, const float4* layer_stats,
                                  float* grad, long long R, int* queue, const int* order,
                                  int persistent, hipStream_t st) {
  const int n_items = tile_end - tile_begin;
  if (n_items <= 0) return hipSuccess;
  const int threads = prm.tile_w * prm.tile_h;
  dim3 grid(persistent ? persistent_grid(n_items, threads) : (unsigned)n_items);
  const size_t lds = (size_t)lds_batch * kRecFloats * sizeof(float);
#define SS_BWD(TW, TH) bwd_t<TW, TH>(grid, lds, st, views, n_views, tile_begin, n_items, ranges, \
                                     sorted_vals, recs, prm, lds_batch, d_image, d_alpha,        \
                                     n_layers, layer_stats, grad, R, queue, order, persistent)
  switch (prm.tile_w * 100 + prm.tile_h) {
    case 808: return SS_BWD(8, 8);
    case 1608: return SS_BWD(16, 8);
    case 1616: return SS_BWD(16, 16);
    case 3208: return SS_BWD(32, 8);
    case 3216: return SS_BWD(32, 16);
    default: return hipErrorInvalidValue;
  }
#undef SS_BWD
}

}  // namespace ss
