// Internal declarations shared by the HIP translation units of libsurfsplat.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ss {

constexpr float kPi = 3.14159265358979323846f;
constexpr int kMaxViews = 64;
constexpr int kMaxLayers = 16;

// ---------------------------------------------------------------- records
// Raster record of one (surfel, view), 16 floats = one 64-byte line.  The
// per-pixel weight uses the projective form of the centre-precomputed MIP
// kernel (eq:mip_weight): with d = (x - x0, y - y0) the pixel offset from the
// projected centre, s = 1 + a3 dx + b3 dy and Q = (M M^T + sigma_f I)^{-1}
// (M = d(x,y)/d(u,v) at the centre), rho^2_mip = d^T Q d / s^2.
enum RecField {
  R_X0 = 0 /* x0 - (i_lo + 1/2) */, R_Y0 /* y0 - (j_lo + 1/2) */, R_QXX, R_QXY2 /* 2 Q_xy */, R_QYY, R_A3, R_B3, R_NF,
  R_ZE, R_CR, R_CG, R_CB, R_RX /* i_lo | i_hi << 16 */, R_RY /* j_lo | j_hi << 16 */,
  R_ZS, R_ID /* record index, as bits */
};
constexpr int kRecFloats = 16;
// Gradient slots per record, written by the raster backward.  Layout
// [R][kGradStride]: the 11 values of one record share one 64-byte line, so the
// atomics a wave issues for one record touch a single line.  Slot G_SS holds
// the densification statistic (sum over pixels of |(dL_p/dT1z, dL_p/dT2z)| T4z,
// Sec. 3.6.1) when it is requested; slot G_TZ the gradient with respect to
// T4z = c'_z through the fragment depths of the depth-consolidation term.
enum GradField { G_X0 = 0, G_Y0, G_QXX, G_QXY2, G_QYY, G_A3, G_B3, G_NF, G_CR, G_CG, G_CB, G_SS, G_TZ };
constexpr int kNGrad = 11;
constexpr int kGradStride = 16;

// What the raster forward leaves for the backward's walk, besides the
// per-layer totals: per pixel the list position (within its group's pair list)
// where each composited layer starts and, at index K, where its walk ended
// (the fragment that would have opened layer K, or 0xffffffff when the list
// ran out), kPosStride words per pixel; and per (tile, 32-record-aligned chunk
// of its list, 4 x 4 quadrant) the 64-bit mask of the chunk's records with a
// fragment accumulated in the quadrant.  Chunk slot of list position p in a
// tile whose list starts at `start`: mask_base + start / 32 + (p - start) / 32 +
// (tile - first tile of the group); distinct (tile, chunk) pairs get distinct
// slots, and a group with pair capacity cap and n tiles needs
// cap / 32 + n + 2 slots of (tile pixels / 16) masks.
constexpr int kPosStride = 17;
struct WalkBufs {
  uint32_t* pos;
  uint64_t* masks;
  long long mask_base;  // first slot of the group
  // deterministic backward: each (record, tile, 8 x 8 sub-tile s) partial goes
  // to sub-slot s of the pair's emission slot,
  // pgrad[((pair_base + offs[inv[record]] + k) * sub_tiles + s) * kGradStride + slot]
  // with k the tile's row-major index in the record's tile rectangle (the
  // order in which the pairs were emitted); null pgrad: float atomics
  float* pgrad;
  const uint32_t* inv;   // global record index -> depth-sorted position in its group
  const uint32_t* offs;  // depth-sorted position -> first emission slot (group-relative)
  long long pair_base;
  // record-major backward: the per-pixel table entries of layers kBwdTabLayers ..
  // kMaxLayers - 1, [pixel][layer - kBwdTabLayers][entry float4s] (the first
  // kBwdTabLayers layers stay in LDS)
  float4* ovf;
};
constexpr int kBwdTabLayers = 8;
inline long long mask_slots(long long pair_cap, int n_tiles) { return pair_cap / 32 + n_tiles + 2; }
// 8 x 8 sub-tiles of a tile (the backward's unit of work)
__host__ __device__ inline int sub_tiles(int tile_w, int tile_h) { return (tile_w / 8) * (tile_h / 8); }

// Long tile lists are split into segments so that no single tile's walk bounds
// a raster launch.  Work item of the persistent raster kernels: (tile, segment,
// segments of the tile, index among the items of split tiles or -1).  A split
// tile's forward runs in three steps: per segment the largest z_end of its
// covering fragments at each pixel, their running maximum over the segments
// (the z_max with which Alg. 1 enters the segment), then the segment walks,
// each recording its own layers -- at most kSegLayers (W, C) totals with their
// fragment counts, and where each began, one more start after them -- which a
// last kernel merges per pixel in list order into the composited result.
constexpr int kSegLayers = 16;
struct SegBufs {
  const int4* items;        // null: one item per tile (order, or tile_begin + item)
  const uint32_t* n_items;  // device count of items
  const int4* mitems;       // the items of split tiles, by their index
  const uint32_t* n_mitems; // device count of those
  int seg_len;              // list entries per segment, a multiple of every LDS batch
  float4* L;                // [mitem][kSegLayers][pixel] local layer (W, C)
  uint16_t* S;              // [mitem][kSegLayers + 1][pixel] local layer start - segment start
  uint16_t* F;              // [mitem][kSegLayers][pixel] fragments of each local layer
  uint32_t* M;              // [mitem][pixel] layers | continues-the-open-layer << 8 | truncated << 9
  float* Z;                 // [mitem][pixel] largest z_end of the segment's covering fragments
  float* ZI;                // [mitem][pixel] largest z_end before the segment (0: none)
};

// ---------------------------------------------------------------- views
struct ViewDev {
  float fx, fy, cx, cy;
  float R[9], t[3];
  float znear;
  float bg[3];
  float cam_o[3];          // camera centre in world space, -R^T t
  int W, H, tiles_x, tiles_y;
  int tile_base;           // global index of the view's first tile
  int scene;
  int n_surf;              // surfels of the scene
  int pad0;
  long long pix_off;       // first pixel of the view in the image arrays
  long long rec_off;       // first record of the view
  long long surf_off;      // first surfel of the scene
  // environment levels: 0 = E, 1..5 specular, 6 = irradiance (split-sum only)
  const float* lvl[7];
  float* dlvl[7];          // their gradients (backward)
  long long* dlvl_fx[7];   // deterministic backward: the same gradients in 64-bit fixed point
  int lh[7], lw[7];
};

struct Params {
  float r_cut, r2, kappa, sigma_f;
  int k_max, shade, tile_w, tile_h;
  const float* lut;
  int lut_nv, lut_r;
  int ss_grad;  // backward: accumulate the screen-space gradient statistic in slot G_SS
  int cons;     // forward: depth statistics (eq:cons_loss, depth image); backward: their adjoint
  int mip;      // 0: centre-precomputed MIP filter; 1: per-pixel Jacobian (forward and backward)
  float t_min;  // transmittance early-out (0: off)
  int tonemap;  // 1: log-space + sRGB transfer of the image (and its derivative in the backward)
  int counters; // forward: count evaluated pairs, fragments, layers and their weight
  int bwd_walk; // backward walk: 1 rows (four records of a quadrant per wave step), 2 record-major
};

// Log-space + sRGB transfer of one linear channel value (the HDR transfer
// used with eq:photo_loss): y = srgb(log(1 + max(x, 0))) with the sRGB
// encoding 12.92 v (v <= 0.0031308) or 1.055 v^(1/2.4) - 0.055, and dy/dx
// (0 for x <= 0).
__device__ __forceinline__ float tonemap_srgb_log(float x) {
  const float v = log1pf(fmaxf(x, 0.f));
  return v <= 0.0031308f ? 12.92f * v : 1.055f * exp2f(log2f(v) * (1.f / 2.4f)) - 0.055f;
}
__device__ __forceinline__ float tonemap_srgb_log_deriv(float x) {
  if (!(x > 0.f)) return 0.f;
  const float v = log1pf(x);
  const float ds = v <= 0.0031308f ? 12.92f : (1.055f / 2.4f) * exp2f(log2f(v) * (1.f / 2.4f - 1.f));
  return ds / (1.f + x);
}

// ---------------------------------------------------------------- FP32 binning
// The binning decision of one (surfel, view): cull, depth-interval start and
// the pixel rectangle that contains the acceptance ellipse {u^T Sigma_mip^{-1}
// u < r_cut^2} (bounding planes tangent to it, App. A.1), widened by 0.01 px.
// Evaluated with a fixed order: no contraction, IEEE division and square root,
// sums left to right.  The same sequence is followed by the CPU reference, so
// keys and rectangles agree bit for bit.
struct Geo {
  float nh[3], uh[3], vh[3];
  float nn, gn, d;
  float tu[3], tv[3];
  float cp[3], up[3], vp[3];
  float z, ez, zs, ze, mx, my, x0, y0;
  float M11, M12, M21, M22, g1, g2, dm, detA;
  int keep;
  int il, ih, jl, jh;  // inclusive pixel rectangle
};

__device__ inline void bin_geometry(const float p[3], const float n[3], const float tg[3],
                                    float su, float sv, const ViewDev& v, float rcut,
                                    float sigma, Geo& o) {
#pragma clang fp contract(off)
  o.keep = 0;
  o.il = 1; o.ih = 0; o.jl = 1; o.jh = 0;
  const float* R = v.R;
  float nn = sqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  float nhx = n[0] / nn, nhy = n[1] / nn, nhz = n[2] / nn;
  float d = tg[0] * nhx + tg[1] * nhy + tg[2] * nhz;
  float gx = tg[0] - d * nhx, gy = tg[1] - d * nhy, gz = tg[2] - d * nhz;
  float gn = sqrtf(gx * gx + gy * gy + gz * gz);
  float ux = gx / gn, uy = gy / gn, uz = gz / gn;
  float vx = nhy * uz - nhz * uy, vy = nhz * ux - nhx * uz, vz = nhx * uy - nhy * ux;
  float tux = su * ux, tuy = su * uy, tuz = su * uz;
  float tvx = sv * vx, tvy = sv * vy, tvz = sv * vz;
  float cpx = R[0] * p[0] + R[1] * p[1] + R[2] * p[2] + v.t[0];
  float cpy = R[3] * p[0] + R[4] * p[1] + R[5] * p[2] + v.t[1];
  float cpz = R[6] * p[0] + R[7] * p[1] + R[8] * p[2] + v.t[2];
  float upx = R[0] * tux + R[1] * tuy + R[2] * tuz;
  float upy = R[3] * tux + R[4] * tuy + R[5] * tuz;
  float upz = R[6] * tux + R[7] * tuy + R[8] * tuz;
  float vpx = R[0] * tvx + R[1] * tvy + R[2] * tvz;
  float vpy = R[3] * tvx + R[4] * tvy + R[5] * tvz;
  float vpz = R[6] * tvx + R[7] * tvy + R[8] * tvz;
  o.nn = nn; o.gn = gn; o.d = d;
  o.nh[0] = nhx; o.nh[1] = nhy; o.nh[2] = nhz;
  o.uh[0] = ux; o.uh[1] = uy; o.uh[2] = uz;
  o.vh[0] = vx; o.vh[1] = vy; o.vh[2] = vz;
  o.tu[0] = tux; o.tu[1] = tuy; o.tu[2] = tuz;
  o.tv[0] = tvx; o.tv[1] = tvy; o.tv[2] = tvz;
  o.cp[0] = cpx; o.cp[1] = cpy; o.cp[2] = cpz;
  o.up[0] = upx; o.up[1] = upy; o.up[2] = upz;
  o.vp[0] = vpx; o.vp[1] = vpy; o.vp[2] = vpz;
  float z = cpz;
  float ez = rcut * sqrtf(upz * upz + vpz * vpz);
  o.z = z; o.ez = ez;
  o.zs = z - ez;
  o.ze = z + ez;
  if (!(z > v.znear)) return;
  float mx = cpx / z, my = cpy / z;
  float x0 = v.fx * mx + v.cx, y0 = v.fy * my + v.cy;
  float M11 = (v.fx * (upx - mx * upz)) / z, M12 = (v.fx * (vpx - mx * vpz)) / z;
  float M21 = (v.fy * (upy - my * upz)) / z, M22 = (v.fy * (vpy - my * vpz)) / z;
  float g1 = upz / z, g2 = vpz / z;
  float dm = M11 * M22 - M12 * M21;
  float detA = dm * dm;
  o.mx = mx; o.my = my; o.x0 = x0; o.y0 = y0;
  o.M11 = M11; o.M12 = M12; o.M21 = M21; o.M22 = M22; o.g1 = g1; o.g2 = g2;
  o.dm = dm; o.detA = detA;
  if (!(detA > 0.f)) return;
  float a = M11 * M11 + M21 * M21, bb = M11 * M12 + M21 * M22, c = M12 * M12 + M22 * M22;
  float S11 = detA + sigma * c, S12 = -(sigma * bb), S22 = detA + sigma * a;
  float Sg1 = S11 * g1 + S12 * g2, Sg2 = S12 * g1 + S22 * g2;
  float gSg = g1 * Sg1 + g2 * Sg2;
  float r2 = rcut * rcut;
  float kz = 1.f - v.znear / z;
  if (!(r2 * gSg < detA * (kz * kz))) return;
  float den = detA - r2 * gSg;
  float SM1x = S11 * M11 + S12 * M12, SM1y = S12 * M11 + S22 * M12;
  float M1SM1 = M11 * SM1x + M12 * SM1y, M1Sg = M11 * Sg1 + M12 * Sg2;
  float SM2x = S11 * M21 + S12 * M22, SM2y = S12 * M21 + S22 * M22;
  float M2SM2 = M21 * SM2x + M22 * SM2y, M2Sg = M21 * Sg1 + M22 * Sg2;
  float Xc = -(r2 * M1Sg) / den;
  float hx = sqrtf(Xc * Xc + (r2 * M1SM1) / den);
  float Yc = -(r2 * M2Sg) / den;
  float hy = sqrtf(Yc * Yc + (r2 * M2SM2) / den);
  float xlo = ((x0 + Xc) - hx) - 0.01f, xhi = ((x0 + Xc) + hx) + 0.01f;
  float ylo = ((y0 + Yc) - hy) - 0.01f, yhi = ((y0 + Yc) + hy) + 0.01f;
  if (!(xlo <= xhi) || !(ylo <= yhi)) return;
  float il = ceilf(xlo - 0.5f), ih = floorf(xhi - 0.5f);
  float jl = ceilf(ylo - 0.5f), jh = floorf(yhi - 0.5f);
  const float wm1 = (float)(v.W - 1), hm1 = (float)(v.H - 1);
  il = (il < 0.f) ? 0.f : il;
  ih = (wm1 < ih) ? wm1 : ih;
  jl = (jl < 0.f) ? 0.f : jl;
  jh = (hm1 < jh) ? hm1 : jh;
  if (!(il <= ih) || !(jl <= jh)) return;
  o.keep = 1;
  o.il = (int)il; o.ih = (int)ih; o.jl = (int)jl; o.jh = (int)jh;
}

// ---------------------------------------------------------------- per fragment
// Evaluation of one record at one pixel, shared by the forward and backward
// raster kernels so that both take identical cutoff decisions: explicit fmaf
// and a fixed order, independent of the surrounding code.
// exp(-q/2) as __expf forms it (the hardware exp2 of its argument times the
// float log2 e), with the two constant factors folded into one: -q/2 and the
// halved constant are exact, so the rounded product, and the result, are the same.
__device__ __forceinline__ float exp_neg_half(float q) {
  return __builtin_amdgcn_exp2f(q * -0.721347510814666748046875f);
}

struct FragEval {
  float dx, dy, s, N, q, w, e;  // e = exp(-q/2), so w = n_f e
  bool cov;
};
__device__ __forceinline__ void frag_eval(const float* rec, int px, int py, float r2, FragEval& f) {
  // R_X0/R_Y0 hold the centre relative to the rectangle's first pixel centre
  const int il = __float_as_int(rec[R_RX]) & 0xffff, jl = __float_as_int(rec[R_RY]) & 0xffff;
  f.dx = (float)(px - il) - rec[R_X0];
  f.dy = (float)(py - jl) - rec[R_Y0];
  f.s = __builtin_fmaf(rec[R_A3], f.dx, __builtin_fmaf(rec[R_B3], f.dy, 1.0f));
  float t = __builtin_fmaf(rec[R_QXX], f.dx, rec[R_QXY2] * f.dy);
  f.N = __builtin_fmaf(t, f.dx, (rec[R_QYY] * f.dy) * f.dy);
  float s2 = f.s * f.s;
  f.cov = f.N < r2 * s2;
  f.q = f.N * __builtin_amdgcn_rcpf(s2);
  f.e = exp_neg_half(f.q);
  f.w = rec[R_NF] * f.e;
}

// Per-pixel-Jacobian variant of the MIP filter (Sec. 3.3.1): J = d(u,v)/d(x,y)
// at this pixel's intersection.  With u = J_c d / s (J_c = M^{-1} at the
// centre, s = 1 + a.d), J = (J_c / s)(I - d a^T / s) and its inverse is
// M_p = s (I + d a^T) M_c, so with B = M_c M_c^T = Q^{-1} - sigma_f I and
// S = M_p M_p^T + sigma_f I:  rho^2 = u^T (I + sigma_f J J^T)^{-1} u = s^2 d^T S^{-1} d
// and n_f = sqrt(det(M_p M_p^T) / det S) = sqrt(s^6 det B / det S), where
// det B = n_f(centre)^2 / det Q avoids the cancellation in Q^{-1} - sigma_f I.
// The support is the binning rectangle intersected with rho^2 < r^2.
__device__ __forceinline__ void frag_eval_pp(const float* rec, int px, int py, float r2, float sigma,
                                             FragEval& f) {
  const int rx = __float_as_int(rec[R_RX]), ry = __float_as_int(rec[R_RY]);
  const int il = rx & 0xffff, ih = rx >> 16, jl = ry & 0xffff, jh = ry >> 16;
  f.dx = (float)(px - il) - rec[R_X0];
  f.dy = (float)(py - jl) - rec[R_Y0];
  const float a3 = rec[R_A3], b3 = rec[R_B3];
  f.s = __builtin_fmaf(a3, f.dx, __builtin_fmaf(b3, f.dy, 1.0f));
  const float qxx = rec[R_QXX], qxy = 0.5f * rec[R_QXY2], qyy = rec[R_QYY];
  const float iq = 1.f / (qxx * qyy - qxy * qxy);
  const float B11 = qyy * iq - sigma, B12 = -qxy * iq, B22 = qxx * iq - sigma;
  const float P11 = 1.f + f.dx * a3, P12 = f.dx * b3, P21 = f.dy * a3, P22 = 1.f + f.dy * b3;
  const float X11 = P11 * B11 + P12 * B12, X12 = P11 * B12 + P12 * B22;
  const float X21 = P21 * B11 + P22 * B12, X22 = P21 * B12 + P22 * B22;
  const float s2 = f.s * f.s;
  const float S11 = s2 * (X11 * P11 + X12 * P12) + sigma;
  const float S12 = s2 * (X11 * P21 + X12 * P22);
  const float S22 = s2 * (X21 * P21 + X22 * P22) + sigma;
  const float detS = S11 * S22 - S12 * S12;
  f.N = s2 * (S22 * f.dx * f.dx - 2.f * S12 * f.dx * f.dy + S11 * f.dy * f.dy);
  const bool in_rect = px >= il && px <= ih && py >= jl && py <= jh;
  f.cov = in_rect && f.s > 0.f && detS > 0.f && f.N < r2 * detS;
  const float idetS = 1.f / detS;  // one division for both uses
  f.q = f.N * idetS;
  const float nfc = rec[R_NF];
  f.e = exp_neg_half(f.q);
  f.w = sqrtf(s2 * s2 * s2 * nfc * nfc * iq * idetS) * f.e;
}

// Adjoint of frag_eval_pp's weight for one fragment: G = w dL/dw (0 for a
// fragment that contributes nothing), written as dL/d(record field) into
// g[G_X0 .. G_NF].  With iq = 1/det Q, B = Q^{-1} - sigma_f I, P = I + d a^T,
// H = P B P^T and S = s^2 H + sigma_f I (the quantities of frag_eval_pp),
//   log w = log n_f + 3 log s + (log iq - log det S)/2 - q/2,
//   q = s^2 (S22 dx^2 - 2 S12 dx dy + S11 dy^2) / det S,
// and the adjoint of H = P B P^T is dL/dP = 2 Gam P B, dL/dB = P^T Gam P with
// Gam the symmetric matrix of dL/dH (off-diagonal halved).  A lane with
// G = 0 evaluates the chain at d = 0 so every output is an exact zero.
__device__ inline void frag_grad_pp(const float* rec, int px, int py, float sigma, float G, bool live,
                                    float* g) {
  const int il = __float_as_int(rec[R_RX]) & 0xffff, jl = __float_as_int(rec[R_RY]) & 0xffff;
  const float dx = live ? (float)(px - il) - rec[R_X0] : 0.f;
  const float dy = live ? (float)(py - jl) - rec[R_Y0] : 0.f;
  const float a3 = rec[R_A3], b3 = rec[R_B3];
  const float s = __builtin_fmaf(a3, dx, __builtin_fmaf(b3, dy, 1.0f));
  const float qxx = rec[R_QXX], qxy = 0.5f * rec[R_QXY2], qyy = rec[R_QYY];
  const float iq = 1.f / (qxx * qyy - qxy * qxy);
  const float B11 = qyy * iq - sigma, B12 = -qxy * iq, B22 = qxx * iq - sigma;
  const float P11 = 1.f + dx * a3, P12 = dx * b3, P21 = dy * a3, P22 = 1.f + dy * b3;
  const float X11 = P11 * B11 + P12 * B12, X12 = P11 * B12 + P12 * B22;
  const float X21 = P21 * B11 + P22 * B12, X22 = P21 * B12 + P22 * B22;
  const float H11 = X11 * P11 + X12 * P12, H12 = X11 * P21 + X12 * P22, H22 = X21 * P21 + X22 * P22;
  const float s2 = s * s;
  const float S11 = s2 * H11 + sigma, S12 = s2 * H12, S22 = s2 * H22 + sigma;
  const float idetS = 1.f / (S11 * S22 - S12 * S12);
  const float Nn = S22 * dx * dx - 2.f * S12 * dx * dy + S11 * dy * dy;
  const float q = s2 * Nn * idetS;
  const float gq = -0.5f * G;                                 // dL/dq
  const float gdet = -(0.5f * G + gq * q) * idetS;            // dL/d det S
  const float gN = gq * s2 * idetS;                           // dL/dNn
  float gs2 = gq * Nn * idetS;
  float gdx = 2.f * gN * (S22 * dx - S12 * dy);
  float gdy = 2.f * gN * (S11 * dy - S12 * dx);
  const float gS11 = gN * dy * dy + gdet * S22;
  const float gS22 = gN * dx * dx + gdet * S11;
  const float gS12 = -2.f * (gN * dx * dy + gdet * S12);
  gs2 += gS11 * H11 + gS12 * H12 + gS22 * H22;
  const float T11 = s2 * gS11, T12 = 0.5f * s2 * gS12, T22 = s2 * gS22;  // Gam
  const float gP11 = 2.f * (T11 * X11 + T12 * X21), gP12 = 2.f * (T11 * X12 + T12 * X22);
  const float gP21 = 2.f * (T12 * X11 + T22 * X21), gP22 = 2.f * (T12 * X12 + T22 * X22);
  const float Y11 = T11 * P11 + T12 * P21, Y12 = T11 * P12 + T12 * P22;
  const float Y21 = T12 * P11 + T22 * P21, Y22 = T12 * P12 + T22 * P22;
  const float gB11 = P11 * Y11 + P21 * Y21, gB12 = 2.f * (P11 * Y12 + P21 * Y22), gB22 = P12 * Y12 + P22 * Y22;
  // B = Q^{-1} - sigma_f I with Q^{-1} = iq [[qyy, -qxy], [-qxy, qxx]]; iq = 1/det Q
  float gqxx = gB22 * iq, gqyy = gB11 * iq, gqxy = -gB12 * iq;
  const float t = -(gB11 * qyy - gB12 * qxy + gB22 * qxx) * iq * iq - 0.5f * G * iq;
  gqxx += t * qyy;
  gqyy += t * qxx;
  gqxy -= 2.f * t * qxy;
  // s = 1 + a . d, P = I + d a^T
  const float gs = 3.f * G * __builtin_amdgcn_rcpf(s) + 2.f * s * gs2;
  gdx += gP11 * a3 + gP12 * b3 + gs * a3;
  gdy += gP21 * a3 + gP22 * b3 + gs * b3;
  g[G_X0] = -gdx;
  g[G_Y0] = -gdy;
  g[G_QXX] = gqxx;
  g[G_QXY2] = 0.5f * gqxy;
  g[G_QYY] = gqyy;
  g[G_A3] = gP11 * dx + gP21 * dy + gs * dx;
  g[G_B3] = gP12 * dx + gP22 * dy + gs * dy;
  g[G_NF] = G / rec[R_NF];
}

__device__ __forceinline__ int view_of_tile(const ViewDev* views, int nv, int tile) {
  int lo = 0, hi = nv - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- launchers
// (implemented in the .hip files; all enqueue on `st` and return hipError_t)
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t st);
hipError_t launch_fill_f32(float* p, float v, long long n, hipStream_t st);
// NaN into p[0..n) when the device status word is SS_ERR_CAPACITY.
hipError_t launch_poison_if_capacity(float* p, long long n, const int* status, hipStream_t st);
// Adds the number of non-finite entries of p[0..n) to *cnt (device).
hipError_t launch_count_nonfinite(const float* p, long long n, unsigned long long* cnt, hipStream_t st);

hipError_t launch_envmap_dirs(float* dirs, int H, int W, hipStream_t st);
hipError_t launch_envmap_out_dirs(int He, int We, const float* in_dirs, const int lh[7],
                                  const int lw[7], float* out_dirs, hipStream_t st);
constexpr int kEnvChunksMax = 64;  // input chunks of the environment prefilter
int envmap_prefilter_chunks(int He, int We);
// part: scratch of envmap_prefilter_chunks(He, We) x (texels of levels 1..6) x 3 floats
hipError_t launch_envmap_prefilter(const float* E, int He, int We, const float* in_dirs,
                                   const float* out_dirs, float* const lvl_out[7], const int lh[7],
                                   const int lw[7], float* part, hipStream_t st);
// status (device): a latched SS_ERR_CAPACITY makes dE NaN.  part (or null):
// deterministic mode, scratch of 3 He We envmap_adjoint_chunks(texels of levels
// 1..6) floats for per-chunk partial sums added in a fixed order.
int envmap_adjoint_chunks(int out_texels);
hipError_t launch_envmap_adjoint(const float* const dlvl[7], const int lh[7], const int lw[7],
                                 const float* out_dirs, int He, int We, const float* in_dirs,
                                 float* dE, const int* status, float* part, hipStream_t st);
hipError_t launch_brdf_lut(float* lut, int n_nv, int n_r, int samples, hipStream_t st);

hipError_t launch_preprocess(const float* const P[7], long long N, const ViewDev* views, int v0,
                             int v1, int max_surf, const Params& prm, float* recs,
                             uint32_t* counts, uint32_t* zkey, uint2* prect, hipStream_t st);
constexpr int kBackwardBlocks = 256;       // blocks of the shading adjoint (per scene): one per CU
constexpr int kBackwardThreads = 512;      // threads per block of the shading adjoint
// LDS budget for privatised environment levels (156 KiB of the 160 KiB per
// CU): with a 128 x 256 map it holds every level but the map itself, so only
// lookups of the sharpest level fall back to global atomics, which are the
// expensive part of the shading adjoint.
constexpr int kLocalMapFloats = 39936;
constexpr int kReduceSplit = 32;           // first-stage chunks of the partial reduction
int backward_blocks(long long n_items);
// fx_exp (device int, or null): deterministic mode; the texel gradients are
// added as integers x 2^(*fx_exp) into the views' dlvl_fx levels (no LDS
// copies: local_total must be 0).
hipError_t launch_shade_backward(const float* const P[7], long long N, const ViewDev* views,
                                 const int* scene_views, int n_scene_views, long long surf_off,
                                 int n_surf, const int local_off[7], int local_total, float* partial,
                                 float* const level_grad[7], const Params& prm, const float* grad,
                                 float* sg, const int* fx_exp, hipStream_t st);
// Deterministic mode: the fixed-point exponent s of a scene, written to *fx_exp
// (after clearing *bound): every texel-gradient contribution of the shading
// adjoint is bounded by 2 max_c |dL/dc_c| max(1, max_c |albedo_c|) of its
// record, and a record adds at most 36 of them, so with s = 61 - ceil(log2(36 n
// bound)) no sum can leave the int64 range.
hipError_t launch_fixed_point_scale(const float* grad, const float* albedo, long long N, const ViewDev* views,
                                    const int* scene_views, int n_scene_views, long long n_surf,
                                    unsigned* bound, int* fx_exp, hipStream_t st);
// dst[i] = src[i] 2^-(*fx_exp) rounded to float, i < n.
hipError_t launch_fixed_to_float(const long long* src, long long n, const int* fx_exp, float* dst, hipStream_t st);
// status (device): a latched SS_ERR_CAPACITY makes every output gradient NaN.
hipError_t launch_geometry_backward(const float* const P[7], long long N, const ViewDev* views,
                                    int n_views, const Params& prm, const float* grad,
                                    const float* sg, float* const G[7], const float* recs,
                                    float* ss_out, int* vis_out, const int* status, hipStream_t st);

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, long long n, uint32_t* total, uint32_t* tmp,
                           long long tmp_n, hipStream_t st);
// Deterministic backward of one group: inv[zidx[i]] = i for the depth order
// zidx of its n records, and, once the raster backward has written the
// per-(record, tile, sub-tile) partials at their emission slots, each record's
// gradient = the sum of its slots in emission order, sub-tiles in order (grad
// rows overwritten).
hipError_t launch_invert_order(const uint32_t* zidx, long long n, uint32_t* inv, hipStream_t st);
hipError_t launch_ordered_record_sums(const uint32_t* zidx, const uint2* zrect, const uint32_t* offs, long long n,
                                      int tile_w, int tile_h, const float* pgrad, long long pair_base,
                                      long long pair_cap, float* grad, hipStream_t st);
// Exclusive scan of the tile counts of record pixel rectangles (il | ih << 16, jl | jh << 16).
hipError_t launch_scan_rect_tiles(const uint2* rect, int tile_w, int tile_h, uint32_t* out, long long n,
                                  uint32_t* total, uint32_t* tmp, long long tmp_n, hipStream_t st);
long long scan_tmp_size(long long n);
hipError_t launch_emit_pairs(const uint32_t* order, const uint2* rect, const uint32_t* offsets,
                             const ViewDev* views, int v0, int v1, long long n_rec, int tile_w, int tile_h,
                             uint32_t* keys, uint32_t* vals, long long cap, int* status, hipStream_t st);
// Stable radix sort of (key, value) pairs over the low first_bits + 8 (passes - 1)
// key bits (first_bits 8, or 9 for a sort without iota values or gather); the
// result is in (keys, vals) for an even pass count, else in the tmp buffers.
// Count: n_fixed when >= 0, else *n_dev (device), at most cap; cap sizes the
// grid and the histogram (radix_hist_size(cap) entries).  iota: the first pass
// takes val0 + position as values.  gsrc (optional): the last pass also writes
// gout[i] = gsrc[value of sorted pair i], or gskip_val where the key is
// gskip_key (gsrc not read there).
long long radix_hist_size(long long cap);
hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                             bool iota, uint32_t val0, const uint2* gsrc, uint2* gout, uint32_t gskip_key,
                             uint2 gskip_val, const uint32_t* n_dev, long long n_fixed, long long cap, int passes,
                             int first_bits, uint32_t* hist, long long hist_n, uint32_t* scan_tmp,
                             long long scan_tmp_n, hipStream_t st);
hipError_t launch_tile_ranges(const uint32_t* keys, const uint32_t* n_pairs, long long cap,
                              uint32_t* ranges, int tile_begin, int n_tiles, hipStream_t st);

// scratch: 66 u32 of device memory (cleared by the call).
hipError_t launch_tile_order(const uint32_t* ranges, int tile_begin, int n_tiles, int* order, uint32_t* scratch,
                             hipStream_t st);
// Work items of a group's raster kernels (persistent launches): every tile in
// `order`; a list longer than max(seg_len, 2 n_pairs / resident tiles) is split
// into segments of seg_len entries (a shorter list's walk ends within about
// the launch's balanced share of the work, so it sets no tail worth the split's
// extra z_max walk and merge).  Resident tiles:
// kResidentWaves forward waves on the chip, one per 8 x 8 sub-tile.  base:
// 2 n_tiles u32 of scratch; counts: 2 u32 (items, items of split tiles); tmp:
// scan scratch.
constexpr uint32_t kResidentWaves = 6144;  // 256 CUs x 4 SIMDs x 6 waves
hipError_t launch_seg_items(const uint32_t* ranges, const int* order, int n_tiles, int seg_len, int tile_pixels,
                            const uint32_t* n_pairs, uint32_t* base, uint32_t* counts, int4* items, int4* mitems,
                            long long items_cap, long long mitems_cap, uint32_t* tmp, long long tmp_n,
                            hipStream_t st);
// n_items: the host's upper bound (grid size); with sb.items the kernels read
// the device count.  With split tiles the forward also runs the z_max steps
// before and the merge after the segment walks.
hipError_t launch_raster_forward(const ViewDev* views, int n_views, int tile_begin, int tile_end,
                                 const uint32_t* ranges, const uint32_t* sorted_vals,
                                 const float* recs, const Params& prm, int lds_batch,
                                 float* image, float* alpha, uint8_t* n_layers_out,
                                 uint8_t* n_layers, float4* layer_stats, float2* layer_stats2,
                                 float* cons, float* depth, int* queue, const int* order,
                                 int persistent, const int* status, unsigned long long* counters,
                                 const WalkBufs& wb, const SegBufs& sb, long long n_items, long long n_mitems,
                                 hipStream_t st);
hipError_t launch_raster_backward(const ViewDev* views, int n_views, int tile_begin, int tile_end,
                                  const uint32_t* ranges, const uint32_t* sorted_vals,
                                  const float* recs, const Params& prm, int lds_batch,
                                  const float* d_image, const float* d_alpha,
                                  const uint8_t* n_layers, const float4* layer_stats,
                                  const float2* layer_stats2, const float* d_cons,
                                  const float* d_depth, float* grad, int* queue,
                                  const int* order, int persistent, const WalkBufs& wb, const SegBufs& sb,
                                  long long n_items, hipStream_t st);

}  // namespace ss
