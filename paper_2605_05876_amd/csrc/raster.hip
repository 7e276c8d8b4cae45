// Tile rasterizer, forward and backward (Alg. 1, eq:shepard, eq:alpha,
// eq:compositing, App. A.1).
//
// Forward: a block owns one tile of TW x TH pixels and each wave64 an 8 x 8
// sub-tile of it, one pixel per lane.  The tile's sorted records are staged
// through LDS in batches (one 64-byte record per surfel, coalesced gathers by
// the whole block).  For each chunk of 64 staged records every lane tests one
// record against the wave's sub-tile (pixel rectangle, then the acceptance
// ellipse), and the wave walks the resulting mask in list order: every lane
// evaluates each surviving record, as Alg. 1 requires.  Per pixel it writes
// the image, alpha, the layer count and each layer's (W_k, C_k)
// (unnormalised), at most K_max of them, the list position where each layer
// starts and where the walk ended, and per (chunk, 4 x 4 quadrant) the mask
// of records that had a fragment accumulated there.
//
// Backward: instead of a replay pass it reads those back (per pixel, never per
// fragment) and rebuilds T_k, alpha_k, C_hat_k and the suffix sums; it takes
// no gap decisions.  One wave per 4 x 4 quadrant steps only the records of the
// quadrant's masks, four at a time (one per 16-lane row), and a lane moves to
// its pixel's next layer when a record's list position reaches that layer's
// recorded start.  Per fragment it forms dL/dw and dL/dc, maps them to the
// record's 11 parameters, reduces them over each row with cross-lane DPP
// moves into the wave's per-record sums in LDS, and after each batch adds
// the waves' sums with one atomic per (record, value) of the tile.
//
// Long tile lists may be split into segments walked in parallel; the
// segment kernels below carry Alg. 1's state across the boundaries.
#include "common.h"

#include <mutex>
#include <vector>

namespace ss {

// Lane -> pixel: wave w owns the 8 x 8 sub-tile (w % (TW/8), w / (TW/8)); row
// r = lane / 16 owns its quadrant (r % 2, r / 2); lane 4 y + x of the row owns
// pixel (x, y) of the quadrant.
template <int TW, int TH>
__device__ __forceinline__ void pixel_of_thread(int t, int tile_x, int tile_y, int& lx, int& ly,
                                                int& sx0, int& sy0) {
  const int lane = t & 63, wave = t >> 6, row = lane >> 4, l16 = lane & 15;
  constexpr int WX = TW / 8;
  const int wx = wave % WX, wy = wave / WX;
  lx = wx * 8 + (row & 1) * 4 + (l16 & 3);
  ly = wy * 8 + (row >> 1) * 4 + (l16 >> 2);
  sx0 = tile_x * TW + wx * 8;
  sy0 = tile_y * TH + wy * 8;
}

// Does the record's pixel rectangle meet the S x S box at (bx, by)?
template <int S>
__device__ __forceinline__ bool rect_meets(const float4 q, int bx, int by) {
  const int rx = __float_as_int(q.x), ry = __float_as_int(q.y);
  const int il = rx & 0xffff, ih = rx >> 16, jl = ry & 0xffff, jh = ry >> 16;
  return !(ih < bx || il > bx + S - 1 || jh < by || jl > by + S - 1);
}

// Stage records vals[b0 .. b0 + cnt) into LDS, 4 threads per record (one
// float4 each).  (Loading all ids first and then all quarters keeps more
// registers live across the walk and was slower.)
template <int NT>
__device__ __forceinline__ void load_batch(float4* lds, const uint32_t* __restrict__ vals,
                                           const float* __restrict__ recs, uint32_t b0, int cnt) {
  for (int j = threadIdx.x; j < cnt * 4; j += NT) {
    const uint32_t id = vals[b0 + (j >> 2)];
    lds[j] = reinterpret_cast<const float4*>(recs + (size_t)id * kRecFloats)[j & 3];
  }
}

// A staged record into registers: the four 16-byte LDS reads are issued
// together, so the walk waits for LDS once per record instead of once for the
// rectangle and again for the fields that depend on it.  NOW: an empty asm
// takes all 16 values, so none of the reads can be sunk into the branches
// that use them (faster in the forward walk, slower in the backward's).
template <bool NOW = false>
__device__ __forceinline__ void load_record(const float4* p, float rec[kRecFloats]) {
  const float4 q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3];
  if constexpr (NOW)
    asm volatile("" ::"v"(q0.x), "v"(q0.y), "v"(q0.z), "v"(q0.w), "v"(q1.x), "v"(q1.y), "v"(q1.z), "v"(q1.w),
                 "v"(q2.x), "v"(q2.y), "v"(q2.z), "v"(q2.w), "v"(q3.x), "v"(q3.y), "v"(q3.z), "v"(q3.w));
  rec[0] = q0.x; rec[1] = q0.y; rec[2] = q0.z; rec[3] = q0.w;
  rec[4] = q1.x; rec[5] = q1.y; rec[6] = q1.z; rec[7] = q1.w;
  rec[8] = q2.x; rec[9] = q2.y; rec[10] = q2.z; rec[11] = q2.w;
  rec[12] = q3.x; rec[13] = q3.y; rec[14] = q3.z; rec[15] = q3.w;
}

// Can the acceptance ellipse of a record reach a pixel centre of the S x S box
// at (bx, by)?  Conservative: with d the pixel offset from the centre,
// rho^2 = d^T Q d / s^2 >= min_box(d^T Q d) / max_box(s)^2, where the minimum of
// the convex quadratic over the box is 0 when the centre is inside and
// otherwise lies on one of its edges (1-D minimum, clamped), and s is linear so
// its maximum is at a corner.  A 1e-3 margin keeps the test far from the
// per-pixel FP32 cutoff decision.
template <int S>
__device__ __forceinline__ bool ellipse_meets(const float4 q0, const float4 q1, const float4 q3,
                                              int bx, int by, float r2) {
  const int il = __float_as_int(q3.x) & 0xffff, jl = __float_as_int(q3.y) & 0xffff;
  const float x0 = (float)(bx - il) - q0.x, x1 = x0 + (float)(S - 1);
  const float y0 = (float)(by - jl) - q0.y, y1 = y0 + (float)(S - 1);
  const float qxx = q0.z, qxy = 0.5f * q0.w, qyy = q1.x, a3 = q1.y, b3 = q1.z;
  const float s00 = 1.f + a3 * x0 + b3 * y0, s01 = 1.f + a3 * x0 + b3 * y1;
  const float s10 = 1.f + a3 * x1 + b3 * y0, s11 = 1.f + a3 * x1 + b3 * y1;
  const float smin = fminf(fminf(s00, s01), fminf(s10, s11));
  const float smax = fmaxf(fmaxf(s00, s01), fmaxf(s10, s11));
  if (!(smin > 0.f)) return true;
  if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return true;
  float nmin = 3.4e38f;
  {
    // the edges' 1-D minimisers by hardware reciprocals: a minimiser off by a
    // relative 1e-7 raises the value found by ~1e-14 of it, far inside the margin
    const float iqyy = __builtin_amdgcn_rcpf(qyy), iqxx = __builtin_amdgcn_rcpf(qxx);
    const float ya = fminf(fmaxf(-qxy * x0 * iqyy, y0), y1), yb = fminf(fmaxf(-qxy * x1 * iqyy, y0), y1);
    nmin = fminf(nmin, qxx * x0 * x0 + 2.f * qxy * x0 * ya + qyy * ya * ya);
    nmin = fminf(nmin, qxx * x1 * x1 + 2.f * qxy * x1 * yb + qyy * yb * yb);
    const float xa = fminf(fmaxf(-qxy * y0 * iqxx, x0), x1), xb = fminf(fmaxf(-qxy * y1 * iqxx, x0), x1);
    nmin = fminf(nmin, qxx * xa * xa + 2.f * qxy * xa * y0 + qyy * y0 * y0);
    nmin = fminf(nmin, qxx * xb * xb + 2.f * qxy * xb * y1 + qyy * y1 * y1);
  }
  return !(nmin >= r2 * smax * smax * 1.001f);
}

// The masks are wave-uniform; saying so keeps them (and the loop over them)
// in scalar registers even though the loop body branches per lane.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Wave-level compaction of a chunk of up to 64 staged records (forward): lane
// j tests record c0 + j against the wave's sub-tile (rectangle, then, for the
// centre MIP filter, the ellipse); the ballot is the (wave-uniform) set of
// records the whole wave visits, in list order.
template <bool ELLIPSE = true>
__device__ __forceinline__ uint64_t chunk_mask(const float4* lds, int c0, int cnt, int lane, int sx0,
                                               int sy0, float r2) {
  const int j = c0 + lane;
  bool ov = false;
  if (j < cnt) {
    const float4 q3 = lds[4 * j + 3];
    ov = rect_meets<8>(q3, sx0, sy0);
    if constexpr (ELLIPSE) ov = ov && ellipse_meets<8>(lds[4 * j], lds[4 * j + 1], q3, sx0, sy0, r2);
  }
  return uniform64(__ballot(ov));
}

__device__ __forceinline__ int next_item(int* queue, int persistent, int& s_item, int iter) {
  if (!persistent) return iter == 0 ? (int)blockIdx.x : -1;
  if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
  __syncthreads();
  int it = s_item;
  __syncthreads();
  return it;
}

// Camera-space depth of the ray-surfel intersection: T4 . (u, v, 1) = T4z / s
// (the perspective denominator s is exactly T4z times an affine function of
// the pixel); T4z = c'_z is the midpoint of the record's depth interval.
__device__ __forceinline__ float frag_depth(const float* rec, const FragEval& f) {
  return 0.5f * (rec[R_ZS] + rec[R_ZE]) / f.s;
}

// Depth statistics of one pixel from its layers (w_k = T_k alpha_k, mean depth
// z_k, depth variance v_k): the depth-consolidation term of eq:cons_loss and
// the composited depth sum_k w_k z_k.
__device__ inline void depth_stats_of_pixel(const float4* __restrict__ st, const float2* __restrict__ st2,
                                            int K, float kappa, float& cons, float& depth) {
  float Ti = 1.f;
  cons = 0.f;
  depth = 0.f;
  for (int i = 0; i < K; ++i) {
    const float Wi = st[i].x, wi = Ti * -expm1f(-kappa * Wi);
    const float2 zi = st2[i];
    float inter = 0.f, Tj = Ti * __expf(-kappa * Wi);
    for (int j = i + 1; j < K; ++j) {
      const float Wj = st[j].x;
      inter += Tj * -expm1f(-kappa * Wj) * fabsf(zi.x - st2[j].x);
      Tj *= __expf(-kappa * Wj);
    }
    cons += wi * (inter + wi * zi.y);
    depth += wi * zi.x;
    Ti *= __expf(-kappa * Wi);
  }
}

// Shepard normalisation of a layer's colour sum: 1/W_k, or 1/|C_k| for the
// normal image (the mean unit normal renormalised to unit length).
__device__ __forceinline__ float layer_norm(int shade, float W, float C0, float C1, float C2) {
  return shade == 2 ? rsqrtf(C0 * C0 + C1 * C1 + C2 * C2) : 1.f / W;
}

// OR over the 16 lanes of a row (DPP: quad swaps, half-row mirror, row mirror).
__device__ __forceinline__ uint32_t row_or(uint32_t x) {
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false);
  return x;
}

// ---------------------------------------------------------------- forward
// CONS: also the per-layer depth statistics (mean, variance; stats2) and the
// per-pixel depth-consolidation term and composited depth (each output
// nullable).  Depths are accumulated relative to the layer's first fragment,
// so the variance does not cancel against z^2.
// PPX: per-pixel-Jacobian MIP filter instead of the centre-precomputed one.
// A latched SS_ERR_CAPACITY in *status (the pair list was cut short) makes
// every pixel NaN.  With prm.counters the kernel adds its work to counters[]:
// (pixel, record) evaluations, accumulated fragments, composited layers (u64)
// and the sum of their weights (f64 in counters[3]).
//
// One work item of the forward: a whole tile (SPLIT false) or one segment of a
// split list (SPLIT true), whose walk records its local layers for the merge
// instead of compositing.  Two instances, so that the plain walk carries none
// of the segment's state.
template <int TW, int TH, bool CONS, bool PPX, bool SPLIT>
__device__ __forceinline__ void forward_item(
    const ViewDev* __restrict__ views, int n_views, int tile_begin, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ vals, const float* __restrict__ recs, const Params& prm, int B,
    float* __restrict__ image, float* __restrict__ alpha, uint8_t* __restrict__ nl_out,
    uint8_t* __restrict__ nl_int, float4* __restrict__ stats, float2* __restrict__ stats2,
    float* __restrict__ cons_out, float* __restrict__ depth_out, bool poisoned,
    unsigned long long* __restrict__ counters, uint32_t* __restrict__ lpos, uint64_t* __restrict__ qmask,
    long long mask_base, const SegBufs& sb, const int4 it) {
  extern __shared__ float4 lds[];
  constexpr int NT = TW * TH;
  constexpr int NQ = TW * TH / 16;  // 4 x 4 quadrants of the tile
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const float r2 = prm.r2, kappa = prm.kappa, t_min = prm.t_min;
  const int kmax = prm.k_max;
  const int tile = it.x;
  constexpr bool split = SPLIT && !CONS;
  const ViewDev& v = views[view_of_tile(views, n_views, tile)];
  const int lt = tile - v.tile_base;
  const int tx = lt % v.tiles_x, ty = lt / v.tiles_x;
  int lx, ly, sx0, sy0;
  pixel_of_thread<TW, TH>(t, tx, ty, lx, ly, sx0, sy0);
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < v.W && py < v.H;
  const long long pix = v.pix_off + (long long)py * v.W + px;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  const uint32_t seg_lo = start + (uint32_t)it.y * (uint32_t)sb.seg_len;
  const uint32_t seg_hi = split ? min(end, seg_lo + (uint32_t)sb.seg_len) : end;
  // split: this pixel's rows of the segment buffers; the largest z_end before
  // the segment is the running z_max of the layer a previous segment left open
  const long long mrow = split ? (long long)it.w * NT + t : 0;
  const long long mlay = split ? (long long)it.w * kSegLayers * NT + t : 0;
  const long long mlayS = split ? (long long)it.w * (kSegLayers + 1) * NT + t : 0;
  const float zin = split ? sb.ZI[mrow] : 0.f;
  bool open_prev = zin > 0.f;
  int Kl = 0, nFl = 0;        // split: local layers closed, fragments of the open one
  bool cont = false, capped = false;

  float C0 = 0.f, C1 = 0.f, C2 = 0.f, Wg = 0.f, zmax = zin;
  float O0 = 0.f, O1 = 0.f, O2 = 0.f, T = 1.f;
  float zr = 0.f, S1 = 0.f, S2 = 0.f;  // CONS: reference depth, sum w dz, sum w dz^2
  int K = 0;
  // r2l: this pixel's cutoff, -inf once its walk has ended (K_max, t_min, a
  // segment's layer cap; outside the view) so that no later fragment covers
  // it.  (A float rather than a flag: the compiler keeps per-lane flags as
  // scalar lane masks and merges them in every branch of the step.)
  float r2l = (!inside || poisoned) ? -__builtin_inff() : r2;
  // list position of the current layer's first fragment (0xffffffff: none yet)
  uint32_t lstart = 0xffffffffu;
  uint32_t* const lp = lpos + pix * kPosStride;
  int nF = 0;              // counters: fragments accumulated by this pixel
  unsigned nE = 0;         // counters: records evaluated at this pixel
  float sumW = 0.f;        // counters: sum of its layers' weights
  // this row's walk mask of chunk slot 0 of the tile (one writer lane per row)
  uint64_t* const qrow = qmask + (mask_base + (start >> 5) + (tile - tile_begin)) * NQ + wave * 4 + (lane >> 4);
  for (uint32_t b0 = seg_lo; b0 < seg_hi; b0 += (uint32_t)B) {
    if (__syncthreads_and(r2l < 0.f)) break;
    const int cnt = (int)min((uint32_t)B, seg_hi - b0);
    load_batch<NT>(lds, vals, recs, b0, cnt);
    __syncthreads();
    for (int c0 = 0; c0 < cnt; c0 += 64) {
      if (__ballot(r2l >= 0.f) == 0ull) break;
      uint64_t m = chunk_mask<!PPX>(lds, c0, cnt, lane, sx0, sy0, r2);
      nE += inside ? (unsigned)__popcll(m) : 0u;
      // the records of the chunk this pixel accumulated; OR-ed over each row of
      // 16 lanes (a 4 x 4 quadrant) they are the backward's walk lists
      // (the two halves of 32 records in turn, so that a step sets its bit in
      // one 32-bit mask)
      uint32_t lm0 = 0u, lm1 = 0u;
      // one record of the chunk at this pixel: its four 16-byte parts, its index
      // b in the chunk, and the mask of its half that records the accumulation
      auto step = [&](const float4 q0, const float4 q1, const float4 q2, const float4 q3, const int b,
                      uint32_t& lm) {
        const uint32_t bit = 1u << (b & 31);  // the record's bit in its half
        const int j = c0 + b;
        const float rec[kRecFloats] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                                       q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
        FragEval f;
        if constexpr (PPX)
          frag_eval_pp(rec, px, py, r2l, prm.sigma_f, f);
        else
          frag_eval(rec, px, py, r2l, f);
        // (structured as nested branches rather than early continues: the
        // compiler then keeps the step's reconvergence simple, which measured
        // faster)
        if (f.cov) {
          if (split && (Wg > 0.f || open_prev) && rec[R_ZS] > zmax) {
            // gap in a segment: close the local layer (if the segment has one open;
            // otherwise this fragment starts a layer after the one a previous
            // segment left open)
            if (Wg > 0.f) {
              sb.L[mlay + (long long)Kl * NT] = make_float4(Wg, C0, C1, C2);
              sb.F[mlay + (long long)Kl * NT] = (uint16_t)nFl;
              ++Kl;
            }
            C0 = C1 = C2 = 0.f;
            Wg = 0.f;
            zmax = 0.f;
            lstart = 0xffffffffu;
            nFl = 0;
            open_prev = false;
            // kSegLayers closed: the layer starting here is beyond K_max globally
            if (Kl >= kSegLayers) {
              r2l = -__builtin_inff();
              capped = true;
              sb.S[mlayS + (long long)kSegLayers * NT] = (uint16_t)(b0 + (uint32_t)j - seg_lo);
            }
          } else if (Wg > 0.f && rec[R_ZS] > zmax) {
            // gap: finalise the layer (Shepard-normalised colour, coverage opacity)
            const float a = -expm1f(-kappa * Wg), e = __expf(-kappa * Wg);
            const float s = T * a * layer_norm(prm.shade, Wg, C0, C1, C2);
            O0 += s * C0; O1 += s * C1; O2 += s * C2;
            stats[pix * kMaxLayers + K] = make_float4(Wg, C0, C1, C2);
            lp[K] = lstart;
            if constexpr (CONS) {
              const float m = S1 / Wg;
              stats2[pix * kMaxLayers + K] = make_float2(zr + m, S2 / Wg - m * m);
              S1 = S2 = 0.f;
            }
            T *= e;
            ++K;
            sumW += Wg;
            C0 = C1 = C2 = 0.f;
            Wg = 0.f;
            zmax = 0.f;
            lstart = 0xffffffffu;
            // K_max cap, or the early-out once the transmittance is below t_min;
            // the discarded fragment's list position ends the pixel's walk
            if (K >= kmax || T < t_min) {
              r2l = -__builtin_inff();
              lp[K] = b0 + (uint32_t)j;
            }
          }
          if (r2l >= 0.f) {
            if constexpr (split) {
              cont = cont || open_prev;  // continues the layer a previous segment left open
              open_prev = false;
              if (lstart == 0xffffffffu) sb.S[mlayS + (long long)Kl * NT] = (uint16_t)(b0 + (uint32_t)j - seg_lo);
              ++nFl;
            }
            // positions increase along the walk and lstart restarts at ~0u per layer
            lstart = min(lstart, b0 + (uint32_t)j);
            lm |= bit;
            if constexpr (CONS) {
              const float z = frag_depth(rec, f);
              if (Wg == 0.f) zr = z;
              const float dz = z - zr;
              S1 += f.w * dz;
              S2 += f.w * dz * dz;
            }
            // depths are positive, so their bit patterns order like the values
            // (one integer max; fmaxf would also canonicalise both operands)
            zmax = __uint_as_float(max(__float_as_uint(rec[R_ZE]), __float_as_uint(zmax)));
            C0 += f.w * rec[R_CR];
            C1 += f.w * rec[R_CG];
            C2 += f.w * rec[R_CB];
            Wg += f.w;
          }
        }
      };
#pragma unroll 1
      for (int h = 0; h < 2; ++h) {
        uint32_t mh = (uint32_t)(m >> (32 * h)), lm = 0u;
        const float4* const lh = lds + 4 * (c0 + 32 * h);
        // two record buffers: the next record's LDS reads are issued before the
        // current one is evaluated, so their latency overlaps the step.  The reads
        // are unconditional (the last step of a half reads its own record again),
        // which keeps the wait for the current record from also waiting for them.
        if (mh) {
          int ba = __builtin_ctz(mh);
          mh &= mh - 1u;
          float4 a0 = lh[4 * ba], a1 = lh[4 * ba + 1], a2 = lh[4 * ba + 2], a3 = lh[4 * ba + 3];
          for (;;) {
            const bool more = mh != 0u;
            const int bn = more ? __builtin_ctz(mh) : ba;
            mh &= mh - 1u;
            const float4 n0 = lh[4 * bn], n1 = lh[4 * bn + 1], n2 = lh[4 * bn + 2], n3 = lh[4 * bn + 3];
            step(a0, a1, a2, a3, 32 * h + ba, lm);
            if (!more) break;
            const bool more2 = mh != 0u;
            ba = more2 ? __builtin_ctz(mh) : bn;
            mh &= mh - 1u;
            a0 = lh[4 * ba]; a1 = lh[4 * ba + 1]; a2 = lh[4 * ba + 2]; a3 = lh[4 * ba + 3];
            step(n0, n1, n2, n3, 32 * h + bn, lm);
            if (!more2) break;
          }
        }
        if (h == 0) lm0 = lm; else lm1 = lm;
      }
      // one bit per fragment this pixel accumulated
      if (prm.counters) nF += __popc(lm0) + __popc(lm1);
      lm0 = row_or(lm0);
      lm1 = row_or(lm1);
      if ((lane & 15) == 0) qrow[(long long)((b0 + (uint32_t)c0 - start) >> 5) * NQ] = ((uint64_t)lm1 << 32) | lm0;
    }
    __syncthreads();
  }
  if (split && inside) {
    if (r2l >= 0.f && Wg > 0.f) {
      sb.L[mlay + (long long)Kl * NT] = make_float4(Wg, C0, C1, C2);
      sb.F[mlay + (long long)Kl * NT] = (uint16_t)nFl;
      ++Kl;
    }
    sb.M[mrow] = (uint32_t)Kl | (cont ? 1u << 8 : 0u) | (capped ? 1u << 9 : 0u);
  } else if (split) {
    sb.M[mrow] = 0u;
  }
  if (!split && inside) {
    if (r2l >= 0.f && Wg > 0.f) {
      const float a = -expm1f(-kappa * Wg), e = __expf(-kappa * Wg);
      const float s = T * a * layer_norm(prm.shade, Wg, C0, C1, C2);
      O0 += s * C0; O1 += s * C1; O2 += s * C2;
      stats[pix * kMaxLayers + K] = make_float4(Wg, C0, C1, C2);
      lp[K] = lstart;
      if constexpr (CONS) {
        const float m = S1 / Wg;
        stats2[pix * kMaxLayers + K] = make_float2(zr + m, S2 / Wg - m * m);
      }
      T *= e;
      ++K;
      sumW += Wg;
    }
    if (r2l >= 0.f) lp[K] = 0xffffffffu;  // the walk ran to the end of the list
    if constexpr (CONS) {
      float cs, dp;
      depth_stats_of_pixel(stats + pix * kMaxLayers, stats2 + pix * kMaxLayers, K, kappa, cs, dp);
      if (cons_out) cons_out[pix] = poisoned ? __builtin_nanf("") : cs;
      if (depth_out) depth_out[pix] = poisoned ? __builtin_nanf("") : dp;
    }
    float o0 = O0 + T * v.bg[0], o1 = O1 + T * v.bg[1], o2 = O2 + T * v.bg[2];
    if (prm.tonemap) {
      o0 = tonemap_srgb_log(o0);
      o1 = tonemap_srgb_log(o1);
      o2 = tonemap_srgb_log(o2);
    }
    float a = 1.f - T;
    if (poisoned) o0 = o1 = o2 = a = __builtin_nanf("");
    image[3 * pix + 0] = o0;
    image[3 * pix + 1] = o1;
    image[3 * pix + 2] = o2;
    alpha[pix] = a;
    nl_int[pix] = (uint8_t)K;
    if (nl_out) nl_out[pix] = (uint8_t)K;
  }
  if (prm.counters) {
    // wave sums, one set of atomics per wave and tile (a split tile's
    // fragments, layers and weights are counted by the merge)
    unsigned long long f = split ? 0u : (unsigned)nF, k = (inside && !split) ? (unsigned)K : 0u, e = nE;
    float w = (inside && !split) ? sumW : 0.f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      f += __shfl_xor(f, off);
      k += __shfl_xor(k, off);
      e += __shfl_xor(e, off);
      w += __shfl_xor(w, off);
    }
    if (lane == 0) {
      if (e) atomicAdd(counters + 0, e);
      if (f) atomicAdd(counters + 1, f);
      if (k) atomicAdd(counters + 2, k);
      if (w != 0.f) atomicAdd(reinterpret_cast<double*>(counters + 3), (double)w);
    }
  }
}

// Occupancy target of the plain variant: 5 waves per SIMD (at most 102 VGPRs:
// the walk holds two staged records; the LDS batches limit a CU to about 5
// waves per SIMD anyway); the compiler's choice for the variants with
// statistics or the per-pixel filter.
template <int TW, int TH, bool CONS, bool PPX>
__global__ void __launch_bounds__(TW* TH)
__attribute__((amdgpu_waves_per_eu((CONS || PPX) ? 1 : 5)))
raster_forward_kernel(
    const ViewDev* __restrict__ views, int n_views, int tile_begin, int n_items,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const float* __restrict__ recs, Params prm, int B, float* __restrict__ image,
    float* __restrict__ alpha, uint8_t* __restrict__ nl_out, uint8_t* __restrict__ nl_int,
    float4* __restrict__ stats, float2* __restrict__ stats2, float* __restrict__ cons_out,
    float* __restrict__ depth_out, int* queue, const int* __restrict__ order, int persistent,
    const int* __restrict__ status, unsigned long long* __restrict__ counters, uint32_t* __restrict__ lpos,
    uint64_t* __restrict__ qmask, long long mask_base, SegBufs sb) {
  __shared__ int s_item;
  const bool poisoned = *status == 3;  // SS_ERR_CAPACITY
  // the items: every tile (in order), or with split lists the tiles and segments
  const int nit = sb.items ? min((int)*sb.n_items, n_items) : n_items;
  for (int iter = 0;; ++iter) {
    const int item = next_item(queue, persistent, s_item, iter);
    if (item < 0 || item >= nit) break;
    const int4 it = sb.items ? sb.items[item] : make_int4(order ? order[item] : tile_begin + item, 0, 1, -1);
    if (!CONS && it.z > 1)
      forward_item<TW, TH, CONS, PPX, true>(views, n_views, tile_begin, ranges, vals, recs, prm, B, image, alpha,
                                            nl_out, nl_int, stats, stats2, cons_out, depth_out, poisoned,
                                            counters, lpos, qmask, mask_base, sb, it);
    else
      forward_item<TW, TH, CONS, PPX, false>(views, n_views, tile_begin, ranges, vals, recs, prm, B, image, alpha,
                                             nl_out, nl_int, stats, stats2, cons_out, depth_out, poisoned,
                                             counters, lpos, qmask, mask_base, sb, it);
  }
}

// ---------------------------------------------------------------- split lists
// Step 1 of a split tile: per segment except the last, the largest z_end of
// the covering fragments at each pixel (the same walk and tests as the
// forward, nothing accumulated).  One block per split item.
template <int TW, int TH, bool PPX>
__device__ __forceinline__ void seg_zmax_item(const ViewDev* __restrict__ views, int n_views,
                                              const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
                                              const float* __restrict__ recs, const Params& prm, int B,
                                              const SegBufs& sb, int m) {
  extern __shared__ float4 lds[];
  constexpr int NT = TW * TH;
  const int4 it = sb.mitems[m];
  if (it.y == it.z - 1) return;  // nothing follows the last segment
  const int t = threadIdx.x, lane = t & 63;
  const ViewDev& v = views[view_of_tile(views, n_views, it.x)];
  const int lt = it.x - v.tile_base;
  const int tx = lt % v.tiles_x, ty = lt / v.tiles_x;
  int lx, ly, sx0, sy0;
  pixel_of_thread<TW, TH>(t, tx, ty, lx, ly, sx0, sy0);
  const int px = tx * TW + lx, py = ty * TH + ly;
  const uint32_t start = ranges[2 * it.x], end = ranges[2 * it.x + 1];
  const uint32_t seg_lo = start + (uint32_t)it.y * (uint32_t)sb.seg_len;
  const uint32_t seg_hi = min(end, seg_lo + (uint32_t)sb.seg_len);
  float zm = 0.f;
  for (uint32_t b0 = seg_lo; b0 < seg_hi; b0 += (uint32_t)B) {
    const int cnt = (int)min((uint32_t)B, seg_hi - b0);
    load_batch<NT>(lds, vals, recs, b0, cnt);
    __syncthreads();
    for (int c0 = 0; c0 < cnt; c0 += 64) {
      uint64_t mk = chunk_mask<!PPX>(lds, c0, cnt, lane, sx0, sy0, prm.r2);
      while (mk) {
        const int j = c0 + __builtin_ctzll(mk);
        mk &= mk - 1;
        float rec[kRecFloats];
        load_record<true>(lds + 4 * j, rec);
        FragEval f;
        if constexpr (PPX)
          frag_eval_pp(rec, px, py, prm.r2, prm.sigma_f, f);
        else
          frag_eval(rec, px, py, prm.r2, f);
        if (f.cov) zm = fmaxf(zm, rec[R_ZE]);
      }
    }
    __syncthreads();
  }
  sb.Z[(long long)m * NT + t] = zm;
}

template <int TW, int TH, bool PPX>
__global__ void __launch_bounds__(TW* TH) seg_zmax_kernel(const ViewDev* __restrict__ views, int n_views,
                                                           const uint32_t* __restrict__ ranges,
                                                           const uint32_t* __restrict__ vals,
                                                           const float* __restrict__ recs, Params prm, int B,
                                                           SegBufs sb, int cap) {
  const int n = min((int)*sb.n_mitems, cap);
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    seg_zmax_item<TW, TH, PPX>(views, n_views, ranges, vals, recs, prm, B, sb, m);
    __syncthreads();  // the item's LDS batches are reused by the next
  }
}

// Step 2: per split tile and pixel, the running maximum over its segments.
// One block per split item; the first segment's block does the tile.
template <int NT>
__global__ void __launch_bounds__(NT) seg_zin_kernel(SegBufs sb, int cap) {
  const int n = min((int)*sb.n_mitems, cap);
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    const int4 it = sb.mitems[m];
    if (it.y != 0) continue;
    const int t = threadIdx.x;
    float z = 0.f;
    for (int k = 0; k < it.z; ++k) {
      sb.ZI[(long long)(m + k) * NT + t] = z;
      if (k + 1 < it.z) z = fmaxf(z, sb.Z[(long long)(m + k) * NT + t]);
    }
  }
}

// Step 4: per split tile and pixel, the segments' local layers merged in list
// order: a segment's first layer joins the layer left open before it when it
// continues that layer; every other local layer is a layer of Alg. 1 (the
// segment entered with the true z_max).  Then the compositing, the K_max cap
// and the early-out, the outputs and the backward's walk record exactly as
// the unsplit forward writes them.
template <int TW, int TH>
__device__ __forceinline__ void seg_merge_item(
    const ViewDev* __restrict__ views, int n_views, const uint32_t* __restrict__ ranges, const Params& prm,
    float* __restrict__ image, float* __restrict__ alpha, uint8_t* __restrict__ nl_out,
    uint8_t* __restrict__ nl_int, float4* __restrict__ stats, const int* __restrict__ status,
    unsigned long long* __restrict__ counters, uint32_t* __restrict__ lpos, const SegBufs& sb, int m0) {
  constexpr int NT = TW * TH;
  const int4 it = sb.mitems[m0];
  if (it.y != 0) return;
  const int t = threadIdx.x, lane = t & 63;
  const ViewDev& v = views[view_of_tile(views, n_views, it.x)];
  const int lt = it.x - v.tile_base;
  const int tx = lt % v.tiles_x, ty = lt / v.tiles_x;
  int lx, ly, sx0, sy0;
  pixel_of_thread<TW, TH>(t, tx, ty, lx, ly, sx0, sy0);
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < v.W && py < v.H;
  const long long pix = v.pix_off + (long long)py * v.W + px;
  const uint32_t start = ranges[2 * it.x];
  const float kappa = prm.kappa, t_min = prm.t_min;
  const int kmax = prm.k_max;
  const bool poisoned = *status == 3;  // SS_ERR_CAPACITY
  uint32_t* const lp = lpos + pix * kPosStride;
  float O0 = 0.f, O1 = 0.f, O2 = 0.f, T = 1.f, sumW = 0.f;
  int K = 0, nF = 0;
  bool done = !inside || poisoned;
  // the open layer: totals, first list position, fragments
  float W = 0.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  uint32_t ls = 0u;
  int lf = 0;
  // finalise the open layer; a layer starting at `next` follows it
  auto close = [&](uint32_t next) {
    const float a = -expm1f(-kappa * W), e = __expf(-kappa * W);
    const float s = T * a * layer_norm(prm.shade, W, C0, C1, C2);
    O0 += s * C0; O1 += s * C1; O2 += s * C2;
    stats[pix * kMaxLayers + K] = make_float4(W, C0, C1, C2);
    lp[K] = ls;
    T *= e;
    ++K;
    sumW += W;
    nF += lf;
    W = 0.f;
    if (K >= kmax || T < t_min) {
      done = true;
      lp[K] = next;
    }
  };
  for (int k = 0; k < it.z && !done; ++k) {
    const long long m = m0 + k;
    const uint32_t meta = sb.M[m * NT + t];
    const int kl = (int)(meta & 255u);
    const bool cont = (meta >> 8) & 1u, capped = (meta >> 9) & 1u;
    const uint32_t seg_lo = start + (uint32_t)k * (uint32_t)sb.seg_len;
    const long long lay = m * kSegLayers * NT + t, layS = m * (kSegLayers + 1) * NT + t;
    for (int j = 0; j < kl && !done; ++j) {
      const float4 L = sb.L[lay + (long long)j * NT];
      const int fj = sb.F[lay + (long long)j * NT];
      if (j == 0 && cont && W > 0.f) {
        W += L.x; C0 += L.y; C1 += L.z; C2 += L.w;
        lf += fj;
        continue;
      }
      const uint32_t sj = seg_lo + sb.S[layS + (long long)j * NT];
      if (W > 0.f) close(sj);
      if (done) break;
      W = L.x; C0 = L.y; C1 = L.z; C2 = L.w;
      ls = sj;
      lf = fj;
    }
    // the segment's walk stopped where its (kSegLayers + 1)-th layer starts,
    // which is past K_max globally
    if (capped && !done) {
      const uint32_t sj = seg_lo + sb.S[layS + (long long)kSegLayers * NT];
      if (W > 0.f) close(sj);
      if (!done) {
        done = true;
        lp[K] = sj;
      }
    }
  }
  if (inside) {
    if (!done && W > 0.f) {
      const float a = -expm1f(-kappa * W), e = __expf(-kappa * W);
      const float s = T * a * layer_norm(prm.shade, W, C0, C1, C2);
      O0 += s * C0; O1 += s * C1; O2 += s * C2;
      stats[pix * kMaxLayers + K] = make_float4(W, C0, C1, C2);
      lp[K] = ls;
      T *= e;
      ++K;
      sumW += W;
      nF += lf;
    }
    if (!done) lp[K] = 0xffffffffu;  // the walk ran to the end of the list
    float o0 = O0 + T * v.bg[0], o1 = O1 + T * v.bg[1], o2 = O2 + T * v.bg[2];
    if (prm.tonemap) {
      o0 = tonemap_srgb_log(o0);
      o1 = tonemap_srgb_log(o1);
      o2 = tonemap_srgb_log(o2);
    }
    float a = 1.f - T;
    if (poisoned) o0 = o1 = o2 = a = __builtin_nanf("");
    image[3 * pix + 0] = o0;
    image[3 * pix + 1] = o1;
    image[3 * pix + 2] = o2;
    alpha[pix] = a;
    nl_int[pix] = (uint8_t)K;
    if (nl_out) nl_out[pix] = (uint8_t)K;
  }
  if (prm.counters) {
    unsigned long long f = inside ? (unsigned)nF : 0u, kk = inside ? (unsigned)K : 0u;
    float w = inside ? sumW : 0.f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      f += __shfl_xor(f, off);
      kk += __shfl_xor(kk, off);
      w += __shfl_xor(w, off);
    }
    if (lane == 0) {
      if (f) atomicAdd(counters + 1, f);
      if (kk) atomicAdd(counters + 2, kk);
      if (w != 0.f) atomicAdd(reinterpret_cast<double*>(counters + 3), (double)w);
    }
  }
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW* TH) seg_merge_kernel(
    const ViewDev* __restrict__ views, int n_views, const uint32_t* __restrict__ ranges, Params prm,
    float* __restrict__ image, float* __restrict__ alpha, uint8_t* __restrict__ nl_out,
    uint8_t* __restrict__ nl_int, float4* __restrict__ stats, const int* __restrict__ status,
    unsigned long long* __restrict__ counters, uint32_t* __restrict__ lpos, SegBufs sb, int cap) {
  const int n = min((int)*sb.n_mitems, cap);
  for (int m = blockIdx.x; m < n; m += gridDim.x)
    seg_merge_item<TW, TH>(views, n_views, ranges, prm, image, alpha, nl_out, nl_int, stats, status, counters,
                           lpos, sb, m);
}

// ---------------------------------------------------------------- backward
// Row-wise transposed reductions: the four 16-lane rows of the wave reduce
// their own values independently (each row carries one record).  A stage
// pairs value a (kept by the lanes whose stage bit is 0) with value b (kept by
// the others): each lane adds its partner's copy across the row (mirror) or
// half-row (half mirror), halving the number of live values; a quad sum
// finishes.  Only DPP moves, no LDS.
__device__ __forceinline__ float dpp_row_mirror(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_half_mirror(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_sum(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
  return x;
}

// 12 values per row: stage 1 (row mirror, lane bit 3) pairs (g_i, g_{i+6}),
// stage 2 (half mirror, lane bit 2) pairs (s_i, s_{i+3}); then quad q of the
// row holds values i + 3q.  Lane 4q + k (k < 3) of a row returns the row total
// of value 3q + k in *vidx, other lanes -1.
__device__ __forceinline__ float row_reduce12(const float g[12], int lane, int* vidx) {
  const bool h8 = (lane & 8) != 0, h4 = (lane & 4) != 0;
  float s[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float keep = h8 ? g[i + 6] : g[i], send = h8 ? g[i] : g[i + 6];
    s[i] = keep + dpp_row_mirror(send);
  }
  float t[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float keep = h4 ? s[i + 3] : s[i], send = h4 ? s[i] : s[i + 3];
    t[i] = quad_sum(keep + dpp_half_mirror(send));
  }
  const int q = (lane >> 2) & 3, k = lane & 3;
  *vidx = k < 3 ? 3 * q + k : -1;
  return k == 0 ? t[0] : (k == 1 ? t[1] : t[2]);
}

// 16 values per row: pairs (g_i, g_{i+8}), then (s_i, s_{i+4}); lane 4q + k of a
// row returns value 4q + k.
__device__ __forceinline__ float row_reduce16(const float g[16], int lane, int* vidx) {
  const bool h8 = (lane & 8) != 0, h4 = (lane & 4) != 0;
  float s[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float keep = h8 ? g[i + 8] : g[i], send = h8 ? g[i] : g[i + 8];
    s[i] = keep + dpp_row_mirror(send);
  }
  float t[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float keep = h4 ? s[i + 4] : s[i], send = h4 ? s[i] : s[i + 4];
    t[i] = quad_sum(keep + dpp_half_mirror(send));
  }
  const int q = (lane >> 2) & 3, k = lane & 3;
  *vidx = 4 * q + k;
  return k == 0 ? t[0] : (k == 1 ? t[1] : (k == 2 ? t[2] : t[3]));
}

// Per-layer coefficients of the backward.  The layer's composited value is
// C_hat = C / W (or C / |C| for the normal image); per fragment
//   dL/dw_f = dW + coef (G' . c_f - GC),  dL/dc_f = w_f coef G',
// with coef = T_k alpha_k / W_k, G' = G and GC = G . C_hat, or, for the
// normal image (C_hat independent of W), G' = (I - C_hat C_hat^T) G W / |C|
// and GC = 0.
struct LayerCoef {
  float W, e, a, Ch0, Ch1, Ch2, dW, coef, GC, G0, G1, G2;
};

__device__ __forceinline__ void layer_coef(const float4 st, float Tk, float kappa, const float G[3],
                                           float ga, float Tfin, const float Cf[3], const float pre[3],
                                           int shade, LayerCoef& L) {
  L.W = st.x;
  L.a = -expm1f(-kappa * st.x);
  L.e = __expf(-kappa * st.x);
  const float iW = 1.f / st.x;
  const float nrm = layer_norm(shade, st.x, st.y, st.z, st.w);
  L.Ch0 = st.y * nrm; L.Ch1 = st.z * nrm; L.Ch2 = st.w * nrm;
  const float ta = Tk * L.a;
  // suffix S_k = sum_{j>k} T_j a_j C_j + T_{K+1} bg = C_final - prefix - T_k a_k C_k
  const float S0 = Cf[0] - pre[0] - ta * L.Ch0;
  const float S1 = Cf[1] - pre[1] - ta * L.Ch1;
  const float S2 = Cf[2] - pre[2] - ta * L.Ch2;
  const float Tk1 = Tk * L.e;
  L.dW = kappa * (G[0] * (Tk1 * L.Ch0 - S0) + G[1] * (Tk1 * L.Ch1 - S1) + G[2] * (Tk1 * L.Ch2 - S2) +
                  ga * Tfin);
  L.coef = ta * iW;
  if (shade == 2) {
    const float gn = G[0] * L.Ch0 + G[1] * L.Ch1 + G[2] * L.Ch2, sc = st.x * nrm;
    L.G0 = (G[0] - gn * L.Ch0) * sc;
    L.G1 = (G[1] - gn * L.Ch1) * sc;
    L.G2 = (G[2] - gn * L.Ch2) * sc;
    L.GC = 0.f;
  } else {
    L.G0 = G[0]; L.G1 = G[1]; L.G2 = G[2];
    L.GC = G[0] * L.Ch0 + G[1] * L.Ch1 + G[2] * L.Ch2;
  }
}

// Adjoint of the depth statistics for layer k of a pixel: loss weight dc on
// the depth-consolidation term and dd on the composited depth, with U the
// running sum over the layers not yet visited of w_i dL/dw_i (2 dc cons + dd
// depth before the first layer).  With
//   dL/dw_k = dc (sum_{j!=k} w_j |z_k - z_j| + 2 w_k v_k) + dd z_k,
//   dL/dz_k = dc w_k sum_{j!=k} w_j sign(z_k - z_j) + dd w_k,  dL/dv_k = dc w_k^2,
// the per-fragment terms are
//   dL/dw_f += A + B (z_f - z_k) + C ((z_f - z_k)^2 - v_k),
//   dL/dz_f  = w_f (B + 2 C (z_f - z_k)),
// A = kappa (T_{k+1} dL/dw_k - sum_{i>k} w_i dL/dw_i) (w_i = T_i alpha_i
// depends on W_k through T_i for i > k), B = dL/dz_k / W_k, C = dL/dv_k / W_k.
struct ConsCoef {
  float A, B, C, z, v;
};
__device__ inline void cons_coef(const float4* __restrict__ st, const float2* __restrict__ st2, int K, int k,
                                 float kappa, float dc, float dd, float& U, ConsCoef& c) {
  const float2 zk = st2[k];
  float T = 1.f, wk = 0.f, Tk1 = 0.f, sabs = 0.f, ssgn = 0.f;
  for (int j = 0; j < K; ++j) {
    const float Wj = st[j].x, e = __expf(-kappa * Wj), wj = T * -expm1f(-kappa * Wj);
    if (j == k) {
      wk = wj;
      Tk1 = T * e;
    } else {
      const float d = zk.x - st2[j].x;
      sabs += wj * fabsf(d);
      ssgn += d > 0.f ? wj : (d < 0.f ? -wj : 0.f);
    }
    T *= e;
  }
  const float dldw = dc * (sabs + 2.f * wk * zk.y) + dd * zk.x;
  U -= dldw * wk;
  c.A = kappa * (dldw * Tk1 - U);
  const float iW = 1.f / st[k].x;
  c.B = wk * (dc * ssgn + dd) * iW;
  c.C = dc * wk * wk * iW;
  c.z = zk.x;
  c.v = zk.y;
}

// The backward works on 8 x 8 sub-tiles of the forward's tiles: one block of
// four waves per (work item, sub-tile), wave q owning the sub-tile's 4 x 4
// quadrant q (walk-mask quadrant 4 s + q of the tile, s the sub-tile in the
// forward's wave order).  It is record-major: the 64 lanes of a wave take the
// records of its quadrant's walk masks, packed across the batch's chunks, and
// loop over the quadrant's 16 pixels together (the pixel uniform across the
// wave), each lane summing its own record's gradient values over the pixels in
// registers; no cross-lane reduction is needed.  A lane finds the layer of its
// fragment by comparing its list position with the pixel's recorded layer
// starts, and reads that layer's coefficients from a per-pixel table the wave
// builds once per work item.
constexpr int kBwdWaves = 4;
constexpr int kBwdThreads = 64 * kBwdWaves;

// The per-pixel table, in float4s: a header {walk end, G (the pixel's dL/dC)}
// and per layer an entry of 1 + normal + 2 cons float4s: {start (layer 0: the
// pixel's layer count), dW, coef, GC}; for the normal image {G' of the layer};
// with the depth statistics {A, B, C, z}, {v}.  The entries of the first
// kBwdTabLayers layers are in LDS, those of deeper layers in global memory
// (WalkBufs::ovf), so that the LDS leaves room for four blocks per CU.
__host__ __device__ constexpr int bwd_entry_floats(bool normal, bool cons) {
  return 4 + (normal ? 4 : 0) + (cons ? 8 : 0);
}
// LDS of a backward block in floats: staged records, the batch's walk masks
// (four quadrants, two floats each), the per-record sums (one set per wave;
// LDS float atomics would cost several cycles per lane), the waves' packed
// record lists (one byte per entry) and the per-pixel tables.  Every part
// starts on a 16-byte boundary.
__host__ __device__ inline size_t bwd_lds_floats(int B, int nv, int lw) {
  return (size_t)B * kRecFloats + (size_t)((B + 63) / 64) * kBwdWaves * 2 + (size_t)kBwdWaves * B * nv +
         (size_t)kBwdWaves * B / 4 + (size_t)kBwdWaves * 16 * (4 + kBwdTabLayers * lw);
}

// The first set bit of a wave-uniform mask (-1 when it is empty), cleared
// from the mask: one scalar find-first-set and one bit clear (a generic ctz
// adds a zero test and a select, m & (m - 1) takes three 64-bit instructions);
// clearing bit -1 of an empty mask (bit 63) leaves it empty.
__device__ __forceinline__ int stake(uint64_t& m) {
  int r;
  asm("s_ff1_i32_b64 %0, %1\n\ts_bitset0_b64 %1, %0" : "=&s"(r), "+s"(m));
  return r;
}
// Two wave-uniform values as the low and high 16-bit halves of one scalar.
__device__ __forceinline__ uint32_t spack16(int lo, int hi) {
  uint32_t r;
  asm("s_pack_ll_b32_b16 %0, %1, %2" : "=s"(r) : "s"(lo), "s"(hi));
  return r;
}

// Set bits of m below this lane.
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// SS: also accumulate the densification statistic in slot G_SS.
// CONS: add the adjoint of the depth statistics (loss weights d_cons on the
// consolidation term, d_depth on the composited depth; either may be null).
// PPX: the per-pixel-Jacobian MIP filter (frag_eval_pp and its adjoint).
// Deterministic mode (wb.pgrad): each (record, sub-tile) sum is stored at the
// pair's emission slot, sub-tile s at sub-slot s; otherwise float atomics.
template <int TW, int TH, bool SS, bool CONS, bool PPX>
__global__ void __launch_bounds__(kBwdThreads)
__attribute__((amdgpu_waves_per_eu((PPX || SS) ? 3 : 4))) raster_backward_records_kernel(
    const ViewDev* __restrict__ views, int n_views, int tile_begin, int n_items,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const float* __restrict__ recs, Params prm, int B, const float* __restrict__ d_image,
    const float* __restrict__ d_alpha, const uint8_t* __restrict__ nl_int,
    const float4* __restrict__ stats, const float2* __restrict__ stats2, const float* __restrict__ d_cons,
    const float* __restrict__ d_depth, float* __restrict__ grad, int* queue,
    const int* __restrict__ order, int persistent, WalkBufs wb, SegBufs sb) {
  constexpr int NSUB = (TW / 8) * (TH / 8);  // 8 x 8 sub-tiles of a tile
  constexpr int NQ = TW * TH / 16;           // walk-mask quadrants of a tile
  constexpr int WX = TW / 8;
  // values summed per record: the 11 record slots, then G_SS, then G_TZ
  constexpr int NV = kNGrad + (SS ? 1 : 0) + (CONS ? 1 : 0);
  constexpr int NT = kBwdThreads;
  // Without the per-fragment statistic or the per-pixel filter, the x0 and y0
  // gradients are linear in per-fragment terms whose record-constant factors
  // come out of the sum: a lane sums the terms and forms them once.
  constexpr bool DEF = !SS && !PPX;
  const uint32_t* __restrict__ lpos = wb.pos;
  const uint64_t* __restrict__ qmask = wb.masks;
  extern __shared__ float4 lds[];
  __shared__ int s_item;
  __shared__ uint32_t s_stop;
  const int t = threadIdx.x, lane = t & 63, q = t >> 6;
  const float r2 = prm.r2, kappa = prm.kappa;
  const bool det = wb.pgrad != nullptr;
  const bool normal = prm.shade == 2;
  const int LW4 = bwd_entry_floats(normal, CONS) / 4;  // float4s per layer entry
  const int pstride = 1 + kBwdTabLayers * LW4;         // float4s per pixel in LDS
  float* const lf = reinterpret_cast<float*>(lds);
  uint64_t* const smask = reinterpret_cast<uint64_t*>(lf + (size_t)B * kRecFloats);  // [chunk][quadrant]
  float* const acc = reinterpret_cast<float*>(smask + ((B + 63) >> 6) * kBwdWaves);
  uint8_t* const lists = reinterpret_cast<uint8_t*>(acc + (size_t)kBwdWaves * B * NV);
  float4* const wtab = reinterpret_cast<float4*>(lists + kBwdWaves * B) + (size_t)q * 16 * pstride;
  uint8_t* const wlist = lists + q * B;
  const int nbase = sb.items ? min((int)*sb.n_items, n_items) : n_items;
  const int nit = nbase * NSUB;
  for (int iter = 0;; ++iter) {
    const int item = next_item(queue, persistent, s_item, iter);
    if (item < 0 || item >= nit) break;
    const int bi = item / NSUB, sub = item - bi * NSUB;
    // a segment of a split list walks its own stretch of the list
    const int4 it = sb.items ? sb.items[bi] : make_int4(order ? order[bi] : tile_begin + bi, 0, 1, -1);
    const int tile = it.x;
    const ViewDev& v = views[view_of_tile(views, n_views, tile)];
    const int lt = tile - v.tile_base;
    const int tx = lt % v.tiles_x, ty = lt / v.tiles_x;
    // this wave's quadrant (as the forward's wave `sub`, row q, laid its pixels out)
    const int qx0 = tx * TW + (sub % WX) * 8 + (q & 1) * 4, qy0 = ty * TH + (sub / WX) * 8 + (q >> 1) * 4;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    const uint32_t seg_lo = start + (uint32_t)it.y * (uint32_t)sb.seg_len;
    const uint32_t seg_hi = it.z > 1 ? min(end, seg_lo + (uint32_t)sb.seg_len) : end;
    if (t == 0) s_stop = seg_lo;
    __syncthreads();

    // The per-pixel table: lane u < 16 takes pixel u = 4 y + x of the quadrant.
    // Entry k: as the forward composited -- transmittance T_k, prefix colour and
    // the suffix through layer_coef, in the order of the layers.
    if (lane < 16) {
      const int px = qx0 + (lane & 3), py = qy0 + (lane >> 2);
      float4* const ph = wtab + lane * pstride;
      uint32_t pend = 0u;
      int nl = 0;
      float G[3] = {0.f, 0.f, 0.f};
      if (px < v.W && py < v.H) {
        const long long pix = v.pix_off + (long long)py * v.W + px;
        G[0] = d_image[3 * pix]; G[1] = d_image[3 * pix + 1]; G[2] = d_image[3 * pix + 2];
        const float ga = d_alpha ? d_alpha[pix] : 0.f;
        nl = nl_int[pix];
        float Cf[3] = {0.f, 0.f, 0.f}, T = 1.f;
        for (int k = 0; k < nl; ++k) {
          const float4 st = stats[pix * kMaxLayers + k];
          const float a = -expm1f(-kappa * st.x), e = __expf(-kappa * st.x);
          const float s = T * a * layer_norm(prm.shade, st.x, st.y, st.z, st.w);
          Cf[0] += s * st.y; Cf[1] += s * st.z; Cf[2] += s * st.w;
          T *= e;
        }
        const float Tfin = T;
        Cf[0] += T * v.bg[0]; Cf[1] += T * v.bg[1]; Cf[2] += T * v.bg[2];
        if (prm.tonemap) {
          // d_image is dL/dy for the tone-mapped y; the walk needs dL/dx
          G[0] *= tonemap_srgb_log_deriv(Cf[0]);
          G[1] *= tonemap_srgb_log_deriv(Cf[1]);
          G[2] *= tonemap_srgb_log_deriv(Cf[2]);
        }
        if (nl > 0) {
          const uint32_t* const lp = lpos + pix * kPosStride;
          pend = lp[nl];
          float dc = 0.f, dd = 0.f, U = 0.f;
          if constexpr (CONS) {
            dc = d_cons ? d_cons[pix] : 0.f;
            dd = d_depth ? d_depth[pix] : 0.f;
            float cs, dp;
            depth_stats_of_pixel(stats + pix * kMaxLayers, stats2 + pix * kMaxLayers, nl, kappa, cs, dp);
            U = 2.f * dc * cs + dd * dp;
          }
          float pre[3] = {0.f, 0.f, 0.f}, Tk = 1.f;
          for (int k = 0; k < nl; ++k) {
            LayerCoef L;
            layer_coef(stats[pix * kMaxLayers + k], Tk, kappa, G, ga, Tfin, Cf, pre, prm.shade, L);
            float4* const e = k < kBwdTabLayers ? ph + 1 + k * LW4
                                                 : wb.ovf + (pix * (kMaxLayers - kBwdTabLayers) + k - kBwdTabLayers) * LW4;
            e[0] = make_float4(k == 0 ? __int_as_float(nl) : __uint_as_float(lp[k]), L.dW, L.coef, L.GC);
            if (normal) e[1] = make_float4(L.G0, L.G1, L.G2, 0.f);
            if constexpr (CONS) {
              ConsCoef CC;
              cons_coef(stats + pix * kMaxLayers, stats2 + pix * kMaxLayers, nl, k, kappa, dc, dd, U, CC);
              e[LW4 - 2] = make_float4(CC.A, CC.B, CC.C, CC.z);
              e[LW4 - 1] = make_float4(CC.v, 0.f, 0.f, 0.f);
            }
            pre[0] += Tk * L.a * L.Ch0; pre[1] += Tk * L.a * L.Ch1; pre[2] += Tk * L.a * L.Ch2;
            Tk *= L.e;
          }
          // the block's batches end where the last of its pixels' walks ended
          atomicMax(&s_stop, pend < end ? pend + 1u : end);
        }
      }
      ph[0] = make_float4(__uint_as_float(pend), G[0], G[1], G[2]);
      if (nl == 0) ph[1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    const uint32_t stop = min(s_stop, seg_hi);
    const long long slot0 = wb.mask_base + (start >> 5) + (tile - tile_begin);
    for (uint32_t b0 = seg_lo; b0 < stop; b0 += (uint32_t)B) {
      const int cnt = (int)min((uint32_t)B, seg_hi - b0);
      const int nch = (cnt + 63) >> 6;
      load_batch<NT>(lds, vals, recs, b0, cnt);
      for (int i = t; i < kBwdWaves * cnt * NV; i += NT) acc[i] = 0.f;
      // the walk masks of the batch's chunks, the sub-tile's four quadrants
      for (int i = t; i < nch * kBwdWaves; i += NT) {
        const int ch = i >> 2, qq = i & 3;
        smask[i] = qmask[(slot0 + ((b0 + (uint32_t)(ch << 6) - start) >> 5)) * NQ + 4 * sub + qq];
      }
      __syncthreads();
      // this wave's records: the set bits of its quadrant's masks, in list order
      // (a wave's LDS operations complete in order, so its lanes read the list
      // back without a barrier).  Bits past the batch are dropped: a chunk the
      // forward did not reach still holds an earlier render's mask.
      int n = 0;
      for (int ch = 0; ch < nch; ++ch) {
        const int left = cnt - (ch << 6);
        const uint64_t m = uniform64(smask[ch * kBwdWaves + q]) & (left >= 64 ? ~0ull : (1ull << left) - 1ull);
        if ((m >> lane) & 1ull) wlist[n + lanes_below(m)] = (uint8_t)(ch * 64 + lane);
        n += __popcll(m);
      }
      for (int e0 = 0; e0 < n; e0 += 64) {
        const bool act = e0 + lane < n;
        const int j = act ? (int)wlist[e0 + lane] : 0;
        float rec[kRecFloats];
        load_record(lds + 4 * j, rec);
        const uint32_t p = b0 + (uint32_t)j;
        const float a3 = rec[R_A3], b3 = rec[R_B3], qxx = rec[R_QXX], qxy2 = rec[R_QXY2], qyy = rec[R_QYY];
        // the pixel offsets from the centre, formed as frag_eval forms them
        const int il = __float_as_int(rec[R_RX]) & 0xffff, jl = __float_as_int(rec[R_RY]) & 0xffff;
        float sum[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) sum[i] = 0.f;
        float svq = 0.f, sgs = 0.f;  // DEF: sums of v and (CONS) of the depth term's s-derivative
        // each pixel's header and first layer (the same address in every lane)
        // are read one pixel ahead, so the LDS latency overlaps the arithmetic
        float4 hd = wtab[0], l0 = wtab[1];
        for (int r = 0; r < 4; ++r) {
          const float dyr = (float)(qy0 + r - jl) - rec[R_Y0];
          const float sb = __builtin_fmaf(b3, dyr, 1.0f), tq = qxy2 * dyr, nq = (qyy * dyr) * dyr;
          for (int c = 0; c < 4; ++c) {
            const float4* const ph = wtab + (4 * r + c) * pstride;
            const float4 hdc = hd, l0c = l0;
            if (4 * r + c < 15) {
              hd = ph[pstride];
              l0 = ph[pstride + 1];
            }
            FragEval f;
            if constexpr (PPX) {
              frag_eval_pp(rec, qx0 + c, qy0 + r, r2, prm.sigma_f, f);
            } else {
              // frag_eval's arithmetic, with the row's terms shared
              f.dx = (float)(qx0 + c - il) - rec[R_X0];
              f.dy = dyr;
              f.s = __builtin_fmaf(a3, f.dx, sb);
              f.N = __builtin_fmaf(__builtin_fmaf(qxx, f.dx, tq), f.dx, nq);
              const float s2 = f.s * f.s;
              f.cov = f.N < r2 * s2;
              f.q = f.N * __builtin_amdgcn_rcpf(s2);
              f.e = exp_neg_half(f.q);
              f.w = rec[R_NF] * f.e;
            }
            if (__ballot(act && f.cov) == 0ull) continue;
            if (act && f.cov && p < __float_as_uint(hdc.x)) {
              // the fragment's layer: the number of the pixel's layer starts at or before p
              // (each table read in its own address space: LDS, or global past kBwdTabLayers)
              const int nl = __float_as_int(l0c.x);
              float4 ev = l0c, gv = l0c, ca = l0c, cb = l0c;
              auto extras = [&](const float4* e) {
                if (normal) gv = e[1];
                if constexpr (CONS) {
                  ca = e[LW4 - 2];
                  cb = e[LW4 - 1];
                }
              };
              if (nl > 1) {
                int k = 0;
                const int nlt = min(nl, kBwdTabLayers);
                for (int kk = 1; kk < nlt; ++kk) k += p >= __float_as_uint(ph[1 + kk * LW4].x) ? 1 : 0;
                // entries of layers past the LDS table: [pixel][layer - kBwdTabLayers]
                const long long db = (v.pix_off + (long long)(qy0 + r) * v.W + qx0 + c) *
                                     (kMaxLayers - kBwdTabLayers) - kBwdTabLayers;
                for (int kk = kBwdTabLayers; kk < nl; ++kk) k += p >= __float_as_uint(wb.ovf[(db + kk) * LW4].x) ? 1 : 0;
                if (k < kBwdTabLayers) {
                  ev = ph[1 + k * LW4];
                  extras(ph + 1 + k * LW4);
                } else {
                  ev = wb.ovf[(db + k) * LW4];
                  extras(wb.ovf + (db + k) * LW4);
                }
              } else {
                extras(ph + 1);
              }
              float G0 = hdc.y, G1 = hdc.z, G2 = hdc.w;
              if (normal) {
                G0 = gv.x; G1 = gv.y; G2 = gv.z;
              }
              const float Gc = G0 * rec[R_CR] + G1 * rec[R_CG] + G2 * rec[R_CB];
              float gw = ev.y + ev.z * (Gc - ev.w);
              const float gcs = f.w * ev.z;
              float gz = 0.f, zf = 0.f;
              if constexpr (CONS) {
                zf = frag_depth(rec, f);
                const float dz = zf - ca.w;
                gw += ca.x + ca.y * dz + ca.z * (dz * dz - cb.x);
                gz = f.w * (ca.y + 2.f * ca.z * dz);
              }
              // d(rho^2)/d(record) for q = d^T Q d / s^2, s = 1 + a3 dx + b3 dy:
              // u = gq / s^2 and v = -2 gq q / s factor every slot of the kernel shape
              const float is = __builtin_amdgcn_rcpf(f.s);
              const float gq = -0.5f * f.w * gw;
              if constexpr (DEF) {
                const float uu = gq * is * is, vq = -2.f * gq * f.q * is;
                const float ux = uu * f.dx, uy = uu * f.dy;
                sum[G_X0] += ux;  // sums of u dx and u dy; x0, y0 after the loop
                sum[G_Y0] += uy;
                svq += vq;
                sum[G_QXX] += ux * f.dx;
                sum[G_QXY2] += ux * f.dy;
                sum[G_QYY] += uy * f.dy;
                sum[G_A3] += vq * f.dx;
                sum[G_B3] += vq * f.dy;
                sum[G_NF] += gw * f.e;  // w / n_f
                sum[G_CR] += gcs * G0;
                sum[G_CG] += gcs * G1;
                sum[G_CB] += gcs * G2;
                if constexpr (CONS) {
                  // z_f = T4z / s: dz/dT4z = 1/s, dz/ds = -z_f/s, ds/d(a3, b3) = (dx, dy),
                  // ds/d(x0, y0) = -(a3, b3)
                  const float gs = -gz * zf * is;
                  sgs += gs;
                  sum[G_A3] += gs * f.dx;
                  sum[G_B3] += gs * f.dy;
                  sum[NV - 1] += gz * is;
                }
              } else {
                float g[NV];
                if constexpr (PPX) {
                  frag_grad_pp(rec, qx0 + c, qy0 + r, prm.sigma_f, f.w * gw, true, g);
                } else {
                  const float uu = gq * is * is, vq = -2.f * gq * f.q * is;
                  const float ux = uu * f.dx, uy = uu * f.dy;
                  g[G_X0] = -(2.f * qxx * ux + qxy2 * uy + a3 * vq);
                  g[G_Y0] = -(qxy2 * ux + 2.f * qyy * uy + b3 * vq);
                  g[G_QXX] = ux * f.dx;
                  g[G_QXY2] = ux * f.dy;
                  g[G_QYY] = uy * f.dy;
                  g[G_A3] = vq * f.dx;
                  g[G_B3] = vq * f.dy;
                  g[G_NF] = gw * f.e;
                }
                g[G_CR] = gcs * G0;
                g[G_CG] = gcs * G1;
                g[G_CB] = gcs * G2;
                if constexpr (CONS) {
                  const float gs = -gz * zf * is;
                  g[G_X0] -= gs * a3;
                  g[G_Y0] -= gs * b3;
                  g[G_A3] += gs * f.dx;
                  g[G_B3] += gs * f.dy;
                  g[NV - 1] = gz * is;
                }
                if constexpr (SS) {
                  // (dL_p/dT1z, dL_p/dT2z) T4z from the record gradients: a change of
                  // T1z (T2z) is the screen map x += delta s / T4z (y += ...), which
                  // moves the centre by delta/T4z and M by E M with E = e1 (a3, b3) / T4z
                  // (e2 ...); the record fields follow in closed form, with
                  // P = I - sigma_f Q and (p1, p2) = (a3, b3) P.
                  const float qxy = 0.5f * qxy2, sg = prm.sigma_f;
                  const float p1 = a3 * (1.f - sg * qxx) - b3 * sg * qxy;
                  const float p2 = b3 * (1.f - sg * qyy) - a3 * sg * qxy;
                  const float gab = a3 * g[G_A3] + b3 * g[G_B3];
                  const float gnf = sg * gw * f.w;  // n_f dL/dn_f sigma_f
                  const float gx = g[G_X0] - 2.f * (qxx * p1 * g[G_QXX] + (qxx * p2 + qxy * p1) * g[G_QXY2] +
                                                    qxy * p2 * g[G_QYY]) -
                                   a3 * gab + gnf * (a3 * qxx + b3 * qxy);
                  const float gy = g[G_Y0] - 2.f * (qxy * p1 * g[G_QXX] + (qxy * p2 + qyy * p1) * g[G_QXY2] +
                                                    qyy * p2 * g[G_QYY]) -
                                   b3 * gab + gnf * (a3 * qxy + b3 * qyy);
                  g[kNGrad] = sqrtf(gx * gx + gy * gy);
                }
#pragma unroll
                for (int i = 0; i < NV; ++i) sum[i] += g[i];
              }
            }
          }
        }
        if constexpr (DEF) {
          const float sux = sum[G_X0], suy = sum[G_Y0];
          sum[G_X0] = -(2.f * qxx * sux + qxy2 * suy + a3 * svq) - a3 * sgs;
          sum[G_Y0] = -(qxy2 * sux + 2.f * qyy * suy + b3 * svq) - b3 * sgs;
        }
        // into the wave's sums for the batch (lanes hold distinct records)
        if (act) {
          float* const a = acc + ((long long)q * cnt + j) * NV;
#pragma unroll
          for (int i = 0; i < NV; ++i) a[i] = sum[i];
        }
      }
      __syncthreads();
      // per (record, value) the waves' sums in a fixed order: one atomic, or
      // (deterministic) a store at the pair's emission slot
      for (int i = t; i < cnt * NV; i += NT) {
        const int j = i / NV, vi = i - j * NV;
        float total = 0.f;
#pragma unroll
        for (int w = 0; w < kBwdWaves; ++w) total += acc[((long long)w * cnt + j) * NV + vi];
        if (total != 0.f) {
          const int slot = vi < kNGrad ? vi : (vi == NV - 1 && CONS ? (int)G_TZ : (int)G_SS);
          const float4 q3 = lds[4 * j + 3];
          const uint32_t id = __float_as_uint(q3.w);
          if (det) {
            const int rx = __float_as_int(q3.x), ry = __float_as_int(q3.y);
            const int tx0 = (rx & 0xffff) / TW, ty0 = (ry & 0xffff) / TH, nx = (rx >> 16) / TW - tx0 + 1;
            const long long e = wb.pair_base + wb.offs[wb.inv[id]] + (ty - ty0) * nx + (tx - tx0);
            wb.pgrad[(e * NSUB + sub) * kGradStride + slot] = total;
          } else {
            atomicAdd(grad + (long long)id * kGradStride + slot, total);
          }
        }
      }
      __syncthreads();
    }
  }
}

// Lane -> pixel of the backward.  A block owns a tile; wave i owns the tile's
// 4 x 4 quadrant(s) numbered as in the forward (quadrant 4 w + r is row r of
// forward wave w).  With up to 16 quadrants a wave owns one and all four rows
// of 16 lanes hold its 16 pixels (R = 4 copies); 32 x 16 tiles (32 quadrants,
// 16 waves) give each wave two, rows 0-1 and 2-3 (R = 2).  Row r of a wave
// takes copy r % R of quadrant r / R.
template <int TW, int TH>
struct BwdMap {
  static constexpr int NQ = TW * TH / 16;           // quadrants per tile
  static constexpr int QW = NQ > 16 ? 2 : 1;        // quadrants per wave
  static constexpr int NW = NQ / QW;                // waves per block
  static constexpr int R = 4 / QW;                  // rows per quadrant
  static constexpr int NT = NW * 64;                // threads per block
};

// The row walk.  SS, CONS, PPX as for the record-major walk; deterministic
// mode stores each (record, tile) sum at sub-slot 0 of the pair's emission slot.
//
// The walk needs no gap tests: the forward recorded where each of a pixel's
// layers starts in the tile list and where its walk ended, and per chunk and
// quadrant which records had a fragment accumulated there.  A wave steps only
// those records, R of them at a time (one per row); a lane's list positions
// increase from step to step, so it advances its layer (transmittance, prefix
// colour and the layer's coefficients, as in the forward's compositing order)
// whenever a position reaches the next layer's start.
// Occupancy target: 5 waves per SIMD (up to 102 VGPRs per lane), 4 with the
// extra statistics or the per-pixel filter.
template <int TW, int TH, bool SS, bool CONS, bool PPX>
__global__ void __launch_bounds__((BwdMap<TW, TH>::NT))
__attribute__((amdgpu_waves_per_eu((SS || CONS || PPX) ? 4 : 5))) raster_backward_rows_kernel(
    const ViewDev* __restrict__ views, int n_views, int tile_begin, int n_items,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const float* __restrict__ recs, Params prm, int B, const float* __restrict__ d_image,
    const float* __restrict__ d_alpha, const uint8_t* __restrict__ nl_int,
    const float4* __restrict__ stats, const float2* __restrict__ stats2, const float* __restrict__ d_cons,
    const float* __restrict__ d_depth, float* __restrict__ grad, int* queue,
    const int* __restrict__ order, int persistent, WalkBufs wb, SegBufs sb) {
  using M = BwdMap<TW, TH>;
  const uint32_t* __restrict__ lpos = wb.pos;
  const uint64_t* __restrict__ qmask = wb.masks;
  const long long mask_base = wb.mask_base;
  // values reduced per fragment: the 11 record slots, then G_SS, then G_TZ
  constexpr int NV = kNGrad + (SS ? 1 : 0) + (CONS ? 1 : 0);
  constexpr int RW = NV <= 12 ? 12 : 16;
  constexpr int NT = M::NT;
  extern __shared__ float4 lds[];
  __shared__ int s_item;
  __shared__ uint32_t s_stop;
  const int t = threadIdx.x, lane = t & 63, row = lane >> 4, wave = t >> 6;
  const int quad = wave * M::QW + row / M::R;       // the tile's quadrant of this lane
  const float r2 = prm.r2, kappa = prm.kappa;
  const int nit = sb.items ? min((int)*sb.n_items, n_items) : n_items;
  for (int iter = 0;; ++iter) {
    const int item = next_item(queue, persistent, s_item, iter);
    if (item < 0 || item >= nit) break;
    // a segment of a split list walks its own stretch of the list; a lane's
    // layer state catches up at its first fragment (the layers' starts are known)
    const int4 it = sb.items ? sb.items[item] : make_int4(order ? order[item] : tile_begin + item, 0, 1, -1);
    const int tile = it.x;
    const ViewDev& v = views[view_of_tile(views, n_views, tile)];
    const int lt = tile - v.tile_base;
    const int tx = lt % v.tiles_x, ty = lt / v.tiles_x;
    int lx, ly, sx0, sy0;
    // the forward's lane of this pixel: wave quad / 4, row quad % 4, same lane in the row
    pixel_of_thread<TW, TH>((quad >> 2) * 64 + (quad & 3) * 16 + (lane & 15), tx, ty, lx, ly, sx0, sy0);
    const int px = tx * TW + lx, py = ty * TH + ly;
    const bool inside = px < v.W && py < v.H;
    const long long pix = v.pix_off + (long long)py * v.W + px;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    const uint32_t seg_lo = start + (uint32_t)it.y * (uint32_t)sb.seg_len;
    const uint32_t seg_hi = it.z > 1 ? min(end, seg_lo + (uint32_t)sb.seg_len) : end;
    if (t == 0) s_stop = seg_lo;
    __syncthreads();

    float G[3] = {0.f, 0.f, 0.f}, ga = 0.f;
    int nl = 0;
    float Cf[3] = {0.f, 0.f, 0.f}, pre[3] = {0.f, 0.f, 0.f};
    float Tfin = 1.f, Tk = 1.f;
    LayerCoef L;
    L.W = 1.f; L.e = 1.f; L.a = 0.f; L.Ch0 = L.Ch1 = L.Ch2 = 0.f; L.dW = 0.f; L.coef = 0.f; L.GC = 0.f;
    L.G0 = L.G1 = L.G2 = 0.f;
    ConsCoef CC;
    CC.A = CC.B = CC.C = CC.z = CC.v = 0.f;
    float dc = 0.f, dd = 0.f, U = 0.f;
    int k = 0;
    uint32_t adv = 0xffffffffu;   // list position where the next layer starts
    uint32_t pend = 0u;           // list position where the pixel's walk ended
    const uint32_t* const lp = lpos + pix * kPosStride;
    if (inside) {
      G[0] = d_image[3 * pix]; G[1] = d_image[3 * pix + 1]; G[2] = d_image[3 * pix + 2];
      ga = d_alpha ? d_alpha[pix] : 0.f;
      nl = nl_int[pix];
      float T = 1.f;
      for (int kk = 0; kk < nl; ++kk) {
        const float4 st = stats[pix * kMaxLayers + kk];
        const float a = -expm1f(-kappa * st.x), e = __expf(-kappa * st.x);
        const float s = T * a * layer_norm(prm.shade, st.x, st.y, st.z, st.w);
        Cf[0] += s * st.y; Cf[1] += s * st.z; Cf[2] += s * st.w;
        T *= e;
      }
      Tfin = T;
      Cf[0] += T * v.bg[0]; Cf[1] += T * v.bg[1]; Cf[2] += T * v.bg[2];
      if (prm.tonemap) {
        // d_image is dL/dy for the tone-mapped y; the walk needs dL/dx
        G[0] *= tonemap_srgb_log_deriv(Cf[0]);
        G[1] *= tonemap_srgb_log_deriv(Cf[1]);
        G[2] *= tonemap_srgb_log_deriv(Cf[2]);
      }
      if (nl > 0) {
        layer_coef(stats[pix * kMaxLayers], 1.f, kappa, G, ga, Tfin, Cf, pre, prm.shade, L);
        if constexpr (CONS) {
          dc = d_cons ? d_cons[pix] : 0.f;
          dd = d_depth ? d_depth[pix] : 0.f;
          float cs, dp;
          depth_stats_of_pixel(stats + pix * kMaxLayers, stats2 + pix * kMaxLayers, nl, kappa, cs, dp);
          U = 2.f * dc * cs + dd * dp;
          cons_coef(stats + pix * kMaxLayers, stats2 + pix * kMaxLayers, nl, 0, kappa, dc, dd, U, CC);
        }
        adv = nl > 1 ? lp[1] : 0xffffffffu;
        pend = lp[nl];
        // the block's batches end where the last of its pixels' walks ended
        atomicMax(&s_stop, pend < end ? pend + 1u : end);
      }
    }
    __syncthreads();
    const uint32_t stop = min(s_stop, seg_hi);
    const long long slot0 = mask_base + (start >> 5) + (tile - tile_begin);
    uint64_t* const smask = reinterpret_cast<uint64_t*>(lds + 4 * B);  // [chunk of the batch][quadrant]
    // per wave, the batch's records' gradient sums [wave][record][value]
    float* const acc = reinterpret_cast<float*>(smask + ((B + 63) >> 6) * M::NQ);
    float* const wacc = acc + (long long)wave * B * NV;
    for (uint32_t b0 = seg_lo; b0 < stop; b0 += (uint32_t)B) {
      const int cnt = (int)min((uint32_t)B, seg_hi - b0);
      load_batch<NT>(lds, vals, recs, b0, cnt);
      for (int i = t; i < M::NW * B * NV; i += NT) acc[i] = 0.f;
      // the walk masks of the batch's chunks, every quadrant of the tile
      const int nch = (cnt + 63) >> 6;
      for (int i = t; i < nch * M::NQ; i += NT) {
        const int ch = i / M::NQ, q = i - ch * M::NQ;
        smask[i] = qmask[(slot0 + ((b0 + (uint32_t)(ch << 6) - start) >> 5)) * M::NQ + q];
      }
      __syncthreads();
      for (int c0 = 0; c0 < cnt; c0 += 64) {
        const uint64_t* qm = smask + (c0 >> 6) * M::NQ + wave * M::QW;
        uint64_t mq0 = uniform64(qm[0]), mq1 = M::QW > 1 ? uniform64(qm[1]) : 0ull;
        while ((mq0 | mq1) != 0ull) {
          // row r takes copy r % R of quadrant r / R: the next R records of its mask
          int jr[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) jr[r] = stake((M::QW > 1 && r >= 2) ? mq1 : mq0);
          // the four record indices as 16-bit halves of two scalars; each lane takes its row's
          const uint32_t p01 = spack16(jr[0], jr[1]), p23 = spack16(jr[2], jr[3]);
          const uint32_t pw = (row & 2) ? p23 : p01;
          const int jl = (int)(short)(pw >> ((row & 1) << 4));
          // idle rows read a valid record and contribute nothing
          float rec[kRecFloats];
          load_record(lds + 4 * (c0 + (jl < 0 ? 0 : jl)), rec);
          FragEval f;
          if constexpr (PPX)
            frag_eval_pp(rec, px, py, r2, prm.sigma_f, f);
          else
            frag_eval(rec, px, py, r2, f);
          bool contrib = false;
          float gw = 0.f, gcs = 0.f, gz = 0.f, zf = 0.f;
          const uint32_t p = b0 + (uint32_t)(c0 + jl);
          if (jl >= 0 && f.cov && p < pend) {
            while (p >= adv) {
              // the fragment lies in a later layer: advance (as the forward composited)
              pre[0] += Tk * L.a * L.Ch0; pre[1] += Tk * L.a * L.Ch1; pre[2] += Tk * L.a * L.Ch2;
              Tk *= L.e;
              ++k;
              layer_coef(stats[pix * kMaxLayers + k], Tk, kappa, G, ga, Tfin, Cf, pre, prm.shade, L);
              if constexpr (CONS)
                cons_coef(stats + pix * kMaxLayers, stats2 + pix * kMaxLayers, nl, k, kappa, dc, dd, U, CC);
              adv = k + 1 < nl ? lp[k + 1] : 0xffffffffu;
            }
            const float Gc = L.G0 * rec[R_CR] + L.G1 * rec[R_CG] + L.G2 * rec[R_CB];
            gw = L.dW + L.coef * (Gc - L.GC);
            gcs = f.w * L.coef;
            if constexpr (CONS) {
              zf = frag_depth(rec, f);
              const float dz = zf - CC.z;
              gw += CC.A + CC.B * dz + CC.C * (dz * dz - CC.v);
              gz = f.w * (CC.B + 2.f * CC.C * dz);
            }
            contrib = true;
          }
          if (__ballot(contrib) == 0ull) continue;
          // d(rho^2)/d(record) for q = d^T Q d / s^2, s = 1 + a3 dx + b3 dy.  Lanes that
          // do not contribute have gw = gcs = gz = 0; zeroing their 1/s, q and w (which
          // may be infinite off the ellipse) makes every value below exactly 0 there.
          const float is = contrib ? __builtin_amdgcn_rcpf(f.s) : 0.f;
          const float fw = contrib ? f.w : 0.f, fe = contrib ? f.e : 0.f;
          const float gq = -0.5f * fw * gw;
          const float dx = f.dx, dy = f.dy, q = contrib ? f.q : 0.f;
          const float qxx = rec[R_QXX], qxy2 = rec[R_QXY2], qyy = rec[R_QYY];
          float g[RW];
          if constexpr (PPX) {
            frag_grad_pp(rec, px, py, prm.sigma_f, fw * gw, contrib, g);
          } else {
            // u = gq / s^2 and v = -2 gq q / s factor every slot of the kernel shape
            const float u = gq * is * is, vq = -2.f * gq * q * is;
            const float ux = u * dx, uy = u * dy;
            g[G_X0] = -(2.f * qxx * ux + qxy2 * uy + rec[R_A3] * vq);
            g[G_Y0] = -(qxy2 * ux + 2.f * qyy * uy + rec[R_B3] * vq);
            g[G_QXX] = ux * dx;
            g[G_QXY2] = ux * dy;
            g[G_QYY] = uy * dy;
            g[G_A3] = vq * dx;
            g[G_B3] = vq * dy;
            g[G_NF] = gw * fe;  // w / n_f
          }
          g[G_CR] = gcs * L.G0;
          g[G_CG] = gcs * L.G1;
          g[G_CB] = gcs * L.G2;
#pragma unroll
          for (int q2 = kNGrad; q2 < RW; ++q2) g[q2] = 0.f;
          if constexpr (CONS) {
            // z_f = T4z / s: dz/dT4z = 1/s, dz/ds = -z_f/s, ds/d(a3, b3) = (dx, dy),
            // ds/d(x0, y0) = -(a3, b3)
            const float gs = -gz * zf * is;
            g[G_X0] -= gs * rec[R_A3];
            g[G_Y0] -= gs * rec[R_B3];
            g[G_A3] += gs * dx;
            g[G_B3] += gs * dy;
            g[NV - 1] = gz * is;
          }
          if constexpr (SS) {
            // (dL_p/dT1z, dL_p/dT2z) T4z from the record gradients: a change of
            // T1z (T2z) is the screen map x += delta s / T4z (y += ...), which moves
            // the centre by delta/T4z and M by E M with E = e1 (a3, b3) / T4z
            // (e2 ...); the record fields follow in closed form, with
            // P = I - sigma_f Q and (p1, p2) = (a3, b3) P.
            const float a3 = rec[R_A3], b3 = rec[R_B3], qxy = 0.5f * qxy2, sg = prm.sigma_f;
            const float p1 = a3 * (1.f - sg * qxx) - b3 * sg * qxy;
            const float p2 = b3 * (1.f - sg * qyy) - a3 * sg * qxy;
            const float gab = a3 * g[G_A3] + b3 * g[G_B3];
            const float gnf = sg * gw * fw;  // n_f dL/dn_f sigma_f
            const float gx = g[G_X0] - 2.f * (qxx * p1 * g[G_QXX] + (qxx * p2 + qxy * p1) * g[G_QXY2] +
                                              qxy * p2 * g[G_QYY]) -
                             a3 * gab + gnf * (a3 * qxx + b3 * qxy);
            const float gy = g[G_Y0] - 2.f * (qxy * p1 * g[G_QXX] + (qxy * p2 + qyy * p1) * g[G_QXY2] +
                                              qyy * p2 * g[G_QYY]) -
                             b3 * gab + gnf * (a3 * qxy + b3 * qyy);
            g[kNGrad] = sqrtf(gx * gx + gy * gy);
          }
          int vidx;
          float tot;
          if constexpr (RW == 12)
            tot = row_reduce12(g, lane, &vidx);
          else
            tot = row_reduce16(g, lane, &vidx);
          // into the wave's sums: with one quadrant per wave the rows hold
          // different records (distinct words); with two, the second quadrant's
          // rows add after the first's (a wave's LDS operations complete in order)
          const bool put = jl >= 0 && vidx >= 0 && vidx < NV && tot != 0.f;
          float* const a = wacc + (c0 + (jl < 0 ? 0 : jl)) * NV + (vidx < 0 ? 0 : vidx);
          if constexpr (M::QW == 1) {
            if (put) *a += tot;
          } else {
            // volatile: the two exclusive per-lane updates must stay two, in order
            volatile float* const va = a;
            if (put && row < 2) *va = *va + tot;
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the first rows' adds are done
            if (put && row >= 2) *va = *va + tot;
          }
        }
      }
      __syncthreads();
      // per (record, value) of the tile, the waves' sums in a fixed order: one
      // atomic, or (deterministic) a store at the pair's emission slot
      for (int i = t; i < cnt * NV; i += NT) {
        const int j = i / NV, vi = i - j * NV;
        float sum = 0.f;
#pragma unroll
        for (int w = 0; w < M::NW; ++w) sum += acc[((long long)w * B + j) * NV + vi];
        if (sum != 0.f) {
          const int slot = vi < kNGrad ? vi : (vi == NV - 1 && CONS ? (int)G_TZ : (int)G_SS);
          const float4 q3 = lds[4 * j + 3];
          const uint32_t id = __float_as_uint(q3.w);
          if (wb.pgrad) {
            const int rx = __float_as_int(q3.x), ry = __float_as_int(q3.y);
            const int tx0 = (rx & 0xffff) / TW, ty0 = (ry & 0xffff) / TH, nx = (rx >> 16) / TW - tx0 + 1;
            const long long e = wb.pair_base + wb.offs[wb.inv[id]] + (ty - ty0) * nx + (tx - tx0);
            wb.pgrad[e * ((TW / 8) * (TH / 8)) * kGradStride + slot] = sum;  // sub-slot 0
          } else {
            atomicAdd(grad + (long long)id * kGradStride + slot, sum);
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- schedule
// Longest-processing-time-first order of a group's tiles for the persistent
// raster: counting sort by bucket floor(log2(list length + 1)) + 1, descending.
// Two kernels: bucket counts (LDS, then one global atomic per bucket and
// block), then placement (each block reserves its run in every bucket with one
// global atomic).  The order inside a bucket depends on block timing; it does
// not matter (it changes only which block renders a tile).
constexpr int kOrderThreads = 256;
constexpr int kOrderBuckets = 33;

__device__ inline int tile_bucket(const uint32_t* ranges, int tile) {
  const uint32_t len = ranges[2 * tile + 1] - ranges[2 * tile];
  return 32 - __clz(len + 1u);
}

__global__ void __launch_bounds__(kOrderThreads) tile_bucket_count_kernel(const uint32_t* __restrict__ ranges,
                                                                          int tile_begin, int n_tiles,
                                                                          uint32_t* __restrict__ counts) {
  __shared__ uint32_t lc[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) lc[threadIdx.x] = 0u;
  __syncthreads();
  const int i = blockIdx.x * kOrderThreads + threadIdx.x;
  if (i < n_tiles) atomicAdd(&lc[tile_bucket(ranges, tile_begin + i)], 1u);
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && lc[threadIdx.x]) atomicAdd(&counts[threadIdx.x], lc[threadIdx.x]);
}

__global__ void __launch_bounds__(kOrderThreads) tile_place_kernel(const uint32_t* __restrict__ ranges,
                                                                   int tile_begin, int n_tiles,
                                                                   const uint32_t* __restrict__ counts,
                                                                   uint32_t* __restrict__ cursor,
                                                                   int* __restrict__ order) {
  __shared__ uint32_t lc[kOrderBuckets], base[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) lc[threadIdx.x] = 0u;
  __syncthreads();
  const int i = blockIdx.x * kOrderThreads + threadIdx.x;
  int b = 0;
  uint32_t rank = 0u;
  if (i < n_tiles) {
    b = tile_bucket(ranges, tile_begin + i);
    rank = atomicAdd(&lc[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && lc[threadIdx.x]) {
    uint32_t start = 0u;  // tiles in longer buckets come first
    for (int k = kOrderBuckets - 1; k > (int)threadIdx.x; --k) start += counts[k];
    base[threadIdx.x] = start + atomicAdd(&cursor[threadIdx.x], lc[threadIdx.x]);
  }
  __syncthreads();
  if (i < n_tiles) order[base[b] + rank] = tile_begin + i;
}

// scratch: 2 * kOrderBuckets u32 (bucket counts and cursors), cleared here.
hipError_t launch_tile_order(const uint32_t* ranges, int tile_begin, int n_tiles, int* order, uint32_t* scratch,
                             hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  hipError_t e = launch_fill_u32(scratch, 0u, 2 * kOrderBuckets, st);
  if (e != hipSuccess) return e;
  const unsigned nb = (unsigned)((n_tiles + kOrderThreads - 1) / kOrderThreads);
  hipLaunchKernelGGL(tile_bucket_count_kernel, dim3(nb), dim3(kOrderThreads), 0, st, ranges, tile_begin, n_tiles,
                     scratch);
  hipLaunchKernelGGL(tile_place_kernel, dim3(nb), dim3(kOrderThreads), 0, st, ranges, tile_begin, n_tiles, scratch,
                     scratch + kOrderBuckets, order);
  return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
// Blocks of a persistent launch: as many as the chip keeps resident at once
// (the kernel's registers and occupancy target, its LDS), at most one per item.
// The occupancy query is cached per (kernel, block, LDS) and not made while the
// stream is being captured; a fixed estimate stands in until it is known.
static unsigned persistent_grid(const void* fn, int n_items, int threads, size_t lds, hipStream_t st) {
  struct Entry {
    const void* fn;
    int threads;
    size_t lds;
    int dev, blocks;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  int dev = 0, blocks = 0;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry& e : cache)
      if (e.fn == fn && e.threads == threads && e.lds == lds && e.dev == dev) blocks = e.blocks;
  }
  if (blocks == 0) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    int cus = 0, per_cu = 0;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) == hipSuccess && cus > 0 &&
        per_cu > 0) {
      blocks = cus * per_cu;
      std::lock_guard<std::mutex> lock(mu);
      cache.push_back(Entry{fn, threads, lds, dev, blocks});
    } else {
      blocks = 256 * (threads <= 64 ? 16 : (threads <= 128 ? 12 : (threads <= 256 ? 8 : 4)));
    }
  }
  return (unsigned)(blocks < n_items ? blocks : (n_items > 0 ? n_items : 1));
}

template <int TW, int TH>
static hipError_t fwd_t(dim3 grid, size_t lds, hipStream_t st, const ViewDev* views, int nv, int tb,
                        int ni, const uint32_t* ranges, const uint32_t* vals, const float* recs,
                        const Params& prm, int B, float* image, float* alpha, uint8_t* nlo,
                        uint8_t* nli, float4* stats, float2* stats2, float* cons, float* depth,
                        int* queue, const int* order, int pers, const int* status,
                        unsigned long long* counters, const WalkBufs& wb, const SegBufs& sb, long long nmi) {
  // split lists: the z_max carried into each segment first
  if (sb.items && nmi > 0) {
    if (prm.mip == 1)
      hipLaunchKernelGGL((seg_zmax_kernel<TW, TH, true>),
                         dim3(persistent_grid(reinterpret_cast<const void*>(&seg_zmax_kernel<TW, TH, true>),
                                              (int)nmi, TW * TH, lds, st)),
                         dim3(TW * TH), lds, st, views, nv,
                         ranges, vals, recs, prm, B, sb, (int)nmi);
    else
      hipLaunchKernelGGL((seg_zmax_kernel<TW, TH, false>),
                         dim3(persistent_grid(reinterpret_cast<const void*>(&seg_zmax_kernel<TW, TH, false>),
                                              (int)nmi, TW * TH, lds, st)),
                         dim3(TW * TH), lds, st, views, nv,
                         ranges, vals, recs, prm, B, sb, (int)nmi);
    hipLaunchKernelGGL((seg_zin_kernel<TW * TH>),
                       dim3(persistent_grid(reinterpret_cast<const void*>(&seg_zin_kernel<TW * TH>), (int)nmi,
                                            TW * TH, 0, st)),
                       dim3(TW * TH), 0, st, sb, (int)nmi);
  }
#define SS_FWD_V(CV, PV)                                                                                   \
  do {                                                                                                      \
    if (pers)                                                                                               \
      grid = dim3(persistent_grid(reinterpret_cast<const void*>(&raster_forward_kernel<TW, TH, CV, PV>), ni, \
                                  TW * TH, lds, st));                                                       \
    hipLaunchKernelGGL((raster_forward_kernel<TW, TH, CV, PV>), grid, dim3(TW * TH), lds, st, views, nv, tb,  \
                       ni, ranges, vals, recs, prm, B, image, alpha, nlo, nli, stats, stats2, cons, depth,    \
                       queue, order, pers, status, counters, wb.pos, wb.masks, wb.mask_base, sb);             \
  } while (0)
  if (prm.mip == 1) {
    if (prm.cons) SS_FWD_V(true, true);
    else SS_FWD_V(false, true);
  } else {
    if (prm.cons) SS_FWD_V(true, false);
    else SS_FWD_V(false, false);
  }
#undef SS_FWD_V
  if (sb.items && nmi > 0)
    hipLaunchKernelGGL((seg_merge_kernel<TW, TH>),
                       dim3(persistent_grid(reinterpret_cast<const void*>(&seg_merge_kernel<TW, TH>), (int)nmi,
                                            TW * TH, 0, st)),
                       dim3(TW * TH), 0, st, views, nv, ranges,
                       prm, image, alpha, nlo, nli, stats, status, counters, wb.pos, sb, (int)nmi);
  return hipGetLastError();
}

template <int TW, int TH, bool SS, bool CONS>
static void bwd_launch(size_t lds, hipStream_t st, const ViewDev* views, int nv, int tb, int ni,
                       const uint32_t* ranges, const uint32_t* vals, const float* recs, const Params& prm,
                       int B, const float* di, const float* da, const uint8_t* nli, const float4* stats,
                       const float2* stats2, const float* dcons, const float* ddepth, float* grad,
                       int* queue, const int* order, int pers, const WalkBufs& wb, const SegBufs& sb) {
  const bool rows = prm.bwd_walk == 1;
  // record-major: one block per (work item, 8 x 8 sub-tile); rows: one per work item
  const int n = rows ? ni : ni * ((TW / 8) * (TH / 8));
  const int threads = rows ? BwdMap<TW, TH>::NT : kBwdThreads;
  const void* fn =
      rows ? (prm.mip == 1 ? reinterpret_cast<const void*>(&raster_backward_rows_kernel<TW, TH, SS, CONS, true>)
                           : reinterpret_cast<const void*>(&raster_backward_rows_kernel<TW, TH, SS, CONS, false>))
           : (prm.mip == 1 ? reinterpret_cast<const void*>(&raster_backward_records_kernel<TW, TH, SS, CONS, true>)
                           : reinterpret_cast<const void*>(&raster_backward_records_kernel<TW, TH, SS, CONS, false>));
  const dim3 grid(pers ? persistent_grid(fn, n, threads, lds, st) : (unsigned)n), block(threads);
#define SS_BWD_K(K, PV)                                                                                     \
  hipLaunchKernelGGL((K<TW, TH, SS, CONS, PV>), grid, block, lds, st, views, nv, tb, ni, ranges, vals, recs, \
                     prm, B, di, da, nli, stats, stats2, dcons, ddepth, grad, queue, order, pers, wb, sb)
  if (rows) {
    if (prm.mip == 1) SS_BWD_K(raster_backward_rows_kernel, true);
    else SS_BWD_K(raster_backward_rows_kernel, false);
  } else {
    if (prm.mip == 1) SS_BWD_K(raster_backward_records_kernel, true);
    else SS_BWD_K(raster_backward_records_kernel, false);
  }
#undef SS_BWD_K
}

template <int TW, int TH>
static hipError_t bwd_t(size_t lds, hipStream_t st, const ViewDev* views, int nv, int tb,
                        int ni, const uint32_t* ranges, const uint32_t* vals, const float* recs,
                        const Params& prm, int B, const float* di, const float* da,
                        const uint8_t* nli, const float4* stats, const float2* stats2, const float* dcons,
                        const float* ddepth, float* grad, int* queue, const int* order,
                        int pers, const WalkBufs& wb, const SegBufs& sb) {
#define SS_BWD_V(SSV, CV) bwd_launch<TW, TH, SSV, CV>(lds, st, views, nv, tb, ni, ranges, vals, recs, \
                                                       prm, B, di, da, nli, stats, stats2, dcons, ddepth, \
                                                       grad, queue, order, pers, wb, sb)
  if (prm.ss_grad && prm.cons) SS_BWD_V(true, true);
  else if (prm.ss_grad) SS_BWD_V(true, false);
  else if (prm.cons) SS_BWD_V(false, true);
  else SS_BWD_V(false, false);
#undef SS_BWD_V
  return hipGetLastError();
}

hipError_t launch_raster_forward(const ViewDev* views, int n_views, int tile_begin, int tile_end,
                                 const uint32_t* ranges, const uint32_t* sorted_vals,
                                 const float* recs, const Params& prm, int lds_batch,
                                 float* image, float* alpha, uint8_t* n_layers_out,
                                 uint8_t* n_layers, float4* layer_stats, float2* layer_stats2,
                                 float* cons, float* depth, int* queue, const int* order,
                                 int persistent, const int* status, unsigned long long* counters,
                                 const WalkBufs& wb, const SegBufs& sb, long long n_items_max, long long n_mitems,
                                 hipStream_t st) {
  const int n_tiles = tile_end - tile_begin;
  if (n_tiles <= 0) return hipSuccess;
  if (prm.cons && (!layer_stats2 || (!cons && !depth))) return hipErrorInvalidValue;
  if (!status || (prm.counters && !counters) || !wb.pos || !wb.masks) return hipErrorInvalidValue;
  // split lists need the persistent queue (the item count is on the device) and no depth statistics
  if (sb.items && (!persistent || prm.cons || !sb.n_items || !sb.mitems || !sb.n_mitems || sb.seg_len <= 0 ||
                   sb.seg_len % lds_batch != 0 || !sb.L || !sb.S || !sb.F || !sb.M || !sb.Z || !sb.ZI))
    return hipErrorInvalidValue;
  const int n_items = sb.items ? (int)n_items_max : n_tiles;
  // persistent launches size their grid per kernel variant
  dim3 grid((unsigned)n_items);
  const size_t lds = (size_t)lds_batch * kRecFloats * sizeof(float);
#define SS_FWD(TW, TH) fwd_t<TW, TH>(grid, lds, st, views, n_views, tile_begin, n_items, ranges, \
                                     sorted_vals, recs, prm, lds_batch, image, alpha,            \
                                     n_layers_out, n_layers, layer_stats, layer_stats2, cons,    \
                                     depth, queue, order, persistent, status, counters, wb, sb,  \
                                     n_mitems)
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
                                  const float2* layer_stats2, const float* d_cons,
                                  const float* d_depth, float* grad, int* queue,
                                  const int* order, int persistent, const WalkBufs& wb, const SegBufs& sb,
                                  long long n_items_max, hipStream_t st) {
  const int n_tiles = tile_end - tile_begin;
  if (n_tiles <= 0) return hipSuccess;
  if (prm.cons && (!layer_stats2 || (!d_cons && !d_depth))) return hipErrorInvalidValue;
  if (!wb.pos || !wb.masks) return hipErrorInvalidValue;
  if (wb.pgrad && (!wb.inv || !wb.offs)) return hipErrorInvalidValue;
  if (sb.items && (!persistent || !sb.n_items || sb.seg_len <= 0 || sb.seg_len % 64 != 0))
    return hipErrorInvalidValue;
  const int n_items = sb.items ? (int)n_items_max : n_tiles;
  if (prm.bwd_walk != 1 && prm.bwd_walk != 2) return hipErrorInvalidValue;
  if (prm.bwd_walk == 2 && !wb.ovf) return hipErrorInvalidValue;
  // The batch shrinks until the block's LDS fits (64 KiB record-major, 120 KiB
  // rows), but not below one 64-record chunk: the forward's walk masks are per
  // chunk of 64 list entries (per 32 when its batch was 32).
  // Record-major: staged records, masks, per-wave sums, record lists, per-pixel
  // tables.  Rows: staged records, the masks of every quadrant, per-wave sums.
  const int nv = kNGrad + (prm.ss_grad ? 1 : 0) + (prm.cons ? 1 : 0);
  const int lw = bwd_entry_floats(prm.shade == 2, prm.cons != 0);
  const int nq = prm.tile_w * prm.tile_h / 16, nw = nq > 16 ? 16 : nq;
  auto lds_for = [&](int b) -> size_t {
    if (prm.bwd_walk == 2) return bwd_lds_floats(b, nv, lw) * sizeof(float);
    return (size_t)b * kRecFloats * sizeof(float) + (size_t)((b + 63) / 64) * nq * sizeof(uint64_t) +
           (size_t)nw * b * nv * sizeof(float);
  };
  const size_t budget = (prm.bwd_walk == 2 ? 64 : 120) * 1024;
  while (lds_batch > 64 && lds_for(lds_batch) > budget) lds_batch /= 2;
  const size_t lds = lds_for(lds_batch);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
#define SS_BWD(TW, TH) bwd_t<TW, TH>(lds, st, views, n_views, tile_begin, n_items, ranges, sorted_vals, recs, \
                                     prm, lds_batch, d_image, d_alpha, n_layers, layer_stats, layer_stats2, \
                                     d_cons, d_depth, grad, queue, order, persistent, wb, sb)
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
