// Per (surfel, view) preprocessing and forward shading, and their adjoint.
//
// Forward (one thread per record): the binning decision (cull, depth interval,
// pixel rectangle; Sec. 3.1, Sec. 3.2.1, App. A.1), the centre-precomputed MIP
// kernel (Sec. 3.3.2) in projective form, and the split-sum colour (eq:ibl).
// Backward: the adjoint of the split-sum colour per record (one thread per
// record; texel gradients into block-private LDS copies of the environment
// levels that fit, wave-cooperative global atomics for the others), then the
// chain rule per surfel (one thread per surfel, looping over the views of its
// scene) from the 11 record gradients written by the raster backward to
// position, normal, tangent, scale, albedo, roughness and metallic.
#include "common.h"

namespace ss {

// Address-space-qualified views of the environment levels: the level pointers
// come from the view descriptors at run time, so without the qualifier every
// texel load and gradient atomic would be a FLAT instruction (and atomics into
// the LDS-privatised levels would take the FLAT path instead of ds_add_f32).
typedef const __attribute__((address_space(1))) float gmem_cf32;
typedef __attribute__((address_space(1))) float gmem_f32;
typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

__device__ __forceinline__ void grad_add(lds_f32* p, float x) {
  __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void grad_add(gmem_f32* p, float x) {
  __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- shading
// NaN maps to 0 so that table indices stay in range
__device__ inline float clamp01(float x) { return !(x >= 0.f) ? 0.f : (x > 1.f ? 1.f : x); }

struct LatLong {
  int r0, r1, c0, c1;
  float fa, fb;
  float th, ph, rho, den;  // for the derivative
};
__device__ inline void latlong_coords(const float d[3], int H, int W, LatLong& L) {
  float rho = sqrtf(d[0] * d[0] + d[1] * d[1]);
  float th = atan2f(rho, d[2]);
  float ph = atan2f(d[1], d[0]);
  if (ph < 0.f) ph += 2.f * kPi;
  // texel scales as products with constant reciprocals (no division per lookup)
  float a = th * ((float)H * (1.f / kPi)) - 0.5f;
  float b = ph * ((float)W * (0.5f / kPi)) - 0.5f;
  if (!(a == a)) a = 0.f;  // NaN direction: any in-range texel
  if (!(b == b)) b = 0.f;
  float a0 = floorf(a), b0 = floorf(b);
  L.fa = a - a0;
  L.fb = b - b0;
  int ia = (int)a0, ib = (int)b0;
  L.r0 = min(max(ia, 0), H - 1);
  L.r1 = min(max(ia + 1, 0), H - 1);
  L.c0 = ((ib % W) + W) % W;
  L.c1 = (L.c0 + 1) % W;
  L.th = th; L.ph = ph; L.rho = rho;
  L.den = rho * rho + d[2] * d[2];
}
__device__ inline void latlong_fetch(const float* mp, int W, const LatLong& L, float out[3]) {
  gmem_cf32* m = (gmem_cf32*)mp;
  gmem_cf32* t00 = m + 3 * (L.r0 * W + L.c0);
  gmem_cf32* t01 = m + 3 * (L.r0 * W + L.c1);
  gmem_cf32* t10 = m + 3 * (L.r1 * W + L.c0);
  gmem_cf32* t11 = m + 3 * (L.r1 * W + L.c1);
  for (int c = 0; c < 3; ++c)
    out[c] = (1.f - L.fa) * ((1.f - L.fb) * t00[c] + L.fb * t01[c]) +
             L.fa * ((1.f - L.fb) * t10[c] + L.fb * t11[c]);
}
struct LutTap { int i0, j0; float fx, fy; };
__device__ inline void lut_fetch(const Params& P, float nv, float r, LutTap& T, float beta[2]) {
  float x = nv * (float)(P.lut_nv - 1), y = r * (float)(P.lut_r - 1);
  T.j0 = min((int)floorf(x), P.lut_nv - 2);
  T.i0 = min((int)floorf(y), P.lut_r - 2);
  T.fx = x - (float)T.j0;
  T.fy = y - (float)T.i0;
  for (int c = 0; c < 2; ++c) {
    float t00 = P.lut[(T.i0 * P.lut_nv + T.j0) * 2 + c];
    float t01 = P.lut[(T.i0 * P.lut_nv + T.j0 + 1) * 2 + c];
    float t10 = P.lut[((T.i0 + 1) * P.lut_nv + T.j0) * 2 + c];
    float t11 = P.lut[((T.i0 + 1) * P.lut_nv + T.j0 + 1) * 2 + c];
    beta[c] = (1.f - T.fy) * ((1.f - T.fx) * t00 + T.fx * t01) + T.fy * ((1.f - T.fx) * t10 + T.fx * t11);
  }
}


// Split-sum colour (eq:ibl): c = k_d rho L_d(n) + L_s(r_dir, r) (F0 beta1 + beta2),
// F0 = 0.04 (1 - m) + rho m, k_d = (1 - F0)(1 - m), r_dir = 2 (w_o.n) n - w_o,
// specular level lambda = 5 r blended linearly between neighbouring levels.
__device__ inline void shade_forward(const ViewDev& v, const Params& P, const float p[3],
                                     const float nh[3], const float rho[3], float rough,
                                     float metal, float col[3]) {
  float wv[3] = {v.cam_o[0] - p[0], v.cam_o[1] - p[1], v.cam_o[2] - p[2]};
  float wl = sqrtf(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
  const float iwl = 1.f / wl;
  float wo[3] = {wv[0] * iwl, wv[1] * iwl, wv[2] * iwl};
  LatLong Li;
  latlong_coords(nh, v.lh[6], v.lw[6], Li);
  float Ld[3];
  latlong_fetch(v.lvl[6], v.lw[6], Li, Ld);
  float nv = nh[0] * wo[0] + nh[1] * wo[1] + nh[2] * wo[2];
  float rd[3] = {2.f * nv * nh[0] - wo[0], 2.f * nv * nh[1] - wo[1], 2.f * nv * nh[2] - wo[2]};
  float rc = clamp01(rough);
  float lam = 5.f * rc;
  int l0 = min((int)floorf(lam), 4);
  float tl = lam - (float)l0;
  LatLong La, Lb;
  latlong_coords(rd, v.lh[l0], v.lw[l0], La);
  latlong_coords(rd, v.lh[l0 + 1], v.lw[l0 + 1], Lb);
  float A[3], B[3];
  latlong_fetch(v.lvl[l0], v.lw[l0], La, A);
  latlong_fetch(v.lvl[l0 + 1], v.lw[l0 + 1], Lb, B);
  LutTap T;
  float beta[2];
  lut_fetch(P, clamp01(nv), rc, T, beta);
  for (int c = 0; c < 3; ++c) {
    float F0 = 0.04f * (1.f - metal) + rho[c] * metal;
    float kd = (1.f - F0) * (1.f - metal);
    float Ls = (1.f - tl) * A[c] + tl * B[c];
    col[c] = kd * rho[c] * Ld[c] + Ls * (F0 * beta[0] + beta[1]);
  }
}

// One bilinear lat-long lookup of the adjoint, split in stages so that a record
// issues the texel loads of all its lookups before it waits for any of them,
// and its gradient atomics only after its last load (a wave's memory counter
// retires in issue order: a load issued after an atomic would wait for it).
//   tap_setup:   coordinates, texel offsets and fractions;
//   tap_fetch:   the 12 texel values;
//   tap_adjoint: the looked-up value, and dL/dd added to gd for g = dL/dvalue;
//   tap_scatter_lds / tap_scatter_global_wave: g times the bilinear weights
//                into the level's LDS copy, or its global gradient map.
struct Tap {
  int o00, o01, o10, o11;  // float offsets of the four texels
  float fa, fb;            // bilinear fractions (row, column)
  float hs, ws;            // H / pi and W / (2 pi)
  float rho, den;          // for the derivative of the coordinates
};
__device__ inline void tap_setup(const float d[3], int H, int W, Tap& T) {
  LatLong L;
  latlong_coords(d, H, W, L);
  T.o00 = 3 * (L.r0 * W + L.c0);
  T.o01 = 3 * (L.r0 * W + L.c1);
  T.o10 = 3 * (L.r1 * W + L.c0);
  T.o11 = 3 * (L.r1 * W + L.c1);
  T.fa = L.fa;
  T.fb = L.fb;
  T.hs = (float)H * (1.f / kPi);
  T.ws = (float)W * (0.5f / kPi);
  T.rho = L.rho;
  T.den = L.den;
}
__device__ inline void tap_fetch(const float* mp, const Tap& T, float t[12]) {
  gmem_cf32* m = (gmem_cf32*)mp;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    t[4 * c + 0] = m[T.o00 + c];
    t[4 * c + 1] = m[T.o01 + c];
    t[4 * c + 2] = m[T.o10 + c];
    t[4 * c + 3] = m[T.o11 + c];
  }
}
__device__ inline void tap_adjoint(const Tap& T, const float t[12], const float d[3], const float g[3],
                                   float val[3], float gd[3]) {
  const float w00 = (1.f - T.fa) * (1.f - T.fb), w01 = (1.f - T.fa) * T.fb;
  const float w10 = T.fa * (1.f - T.fb), w11 = T.fa * T.fb;
  float ga = 0.f, gb = 0.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float v00 = t[4 * c], v01 = t[4 * c + 1], v10 = t[4 * c + 2], v11 = t[4 * c + 3];
    val[c] = w00 * v00 + w01 * v01 + w10 * v10 + w11 * v11;
    ga += g[c] * ((1.f - T.fb) * (v10 - v00) + T.fb * (v11 - v01));
    gb += g[c] * ((1.f - T.fa) * (v01 - v00) + T.fa * (v11 - v10));
  }
  const float gth = ga * T.hs, gph = gb * T.ws;
  if (T.rho > 1e-20f && T.den > 0.f) {
    // th = atan2(rho, z), ph = atan2(y, x), rho = sqrt(x^2 + y^2)
    const float iden = 1.f / T.den, irho = 1.f / T.rho;
    const float dth_drho = d[2] * iden, dth_dz = -T.rho * iden;
    const float a = gth * dth_drho * irho, b = gph * irho * irho;
    gd[0] += a * d[0] - b * d[1];
    gd[1] += a * d[1] + b * d[0];
    gd[2] += gth * dth_dz;
  }
}
// Texel gradients g times the bilinear weights.  Global maps take float
// atomics.  Into an LDS copy, a float atomic add serialises the lanes of a
// wave (about 3 cycles per lane on this part) while a 32-bit compare-and-swap
// runs at close to the integer atomic rate: every lane first reads its twelve
// words, then tries one compare-and-swap per word (new = old + x, the same
// IEEE sum an atomic add forms), and only the lanes whose attempt lost a race
// (another lane or wave wrote the word in between) fall back to the atomic add.
__device__ __forceinline__ void tap_weights(const Tap& T, float w[4]) {
  w[0] = (1.f - T.fa) * (1.f - T.fb);
  w[1] = (1.f - T.fa) * T.fb;
  w[2] = T.fa * (1.f - T.fb);
  w[3] = T.fa * T.fb;
}
__device__ inline void tap_scatter_lds(lds_f32* dm, const Tap& T, const float g[3]) {
  float w[4];
  tap_weights(T, w);
  const int o[4] = {T.o00, T.o01, T.o10, T.o11};
  lds_u32* a[12];
  float x[12];
  uint32_t old[12];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[4 * c + k] = (lds_u32*)(dm + o[k] + c);
      x[4 * c + k] = g[c] * w[k];
    }
#pragma unroll
  for (int i = 0; i < 12; ++i)
    old[i] = x[i] != 0.f ? __hip_atomic_load(a[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0u;
  bool lost[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    lost[i] = false;
    if (x[i] != 0.f) {
      uint32_t e = old[i];
      lost[i] = !__hip_atomic_compare_exchange_strong(a[i], &e, __float_as_uint(__uint_as_float(old[i]) + x[i]),
                                                      __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
#pragma unroll
  for (int i = 0; i < 12; ++i)
    if (lost[i]) grad_add((lds_f32*)a[i], x[i]);
}
// Texel gradients into a global map, by the whole wave: the lanes with a
// global lookup are taken one at a time, and lanes 0..11 each add one of that
// lookup's twelve values (tap k / 3, channel k % 3).  One atomic instruction
// then covers the lookup's two runs of six consecutive floats (one or two
// cache lines) instead of twelve instructions that each touch a different line
// per lane: the L2 processes float atomics per (instruction, cache line), and
// scattered ones ran at about 21 G lanes/s on this part.  Called by every lane
// of the wave; `mine` says whether this lane has a lookup to scatter.
__device__ inline void tap_scatter_global_wave(bool mine, float* dm, const Tap& T, const float g[3]) {
  const int lane = (int)(threadIdx.x & 63);
  const int tap = lane / 3, c = lane - 3 * tap;
  // (readfirstlane returns int: both halves go through uint32_t, so the low
  // half is not sign-extended into the lanes 32..63 of the mask)
  const uint64_t bal = __ballot(mine);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)bal);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(bal >> 32));
  uint64_t m = ((uint64_t)hi << 32) | lo;
  const uint64_t pd = (uint64_t)(uintptr_t)dm;
  while (m) {
    const int src = (int)__builtin_ctzll(m);
    m &= m - 1;
    const uint64_t base = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(pd >> 32), src) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)pd, src);
    const int o0 = __builtin_amdgcn_readlane(T.o00, src), o1 = __builtin_amdgcn_readlane(T.o01, src);
    const int o2 = __builtin_amdgcn_readlane(T.o10, src), o3 = __builtin_amdgcn_readlane(T.o11, src);
    const float fa = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(T.fa), src));
    const float fb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(T.fb), src));
    const float g0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g[0]), src));
    const float g1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g[1]), src));
    const float g2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g[2]), src));
    if (lane < 12) {
      const int o = tap == 0 ? o0 : (tap == 1 ? o1 : (tap == 2 ? o2 : o3));
      const float wa = tap < 2 ? 1.f - fa : fa, wb = (tap & 1) ? fb : 1.f - fb;
      const float x = (c == 0 ? g0 : (c == 1 ? g1 : g2)) * (wa * wb);
      if (x != 0.f) grad_add((gmem_f32*)(uintptr_t)base + o + c, x);
    }
  }
}

// Deterministic variant of tap_scatter_global_wave: the same cooperative walk
// over the wave's lookups, each value added as the 64-bit integer
// round(x 2^s) (integer sums do not depend on their order).
__device__ inline void tap_scatter_global_wave_fx(bool mine, long long* dm, const Tap& T, const float g[3],
                                                  double scale) {
  const int lane = (int)(threadIdx.x & 63);
  const int tap = lane / 3, c = lane - 3 * tap;
  const uint64_t bal = __ballot(mine);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)bal);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(bal >> 32));
  uint64_t m = ((uint64_t)hi << 32) | lo;
  const uint64_t pd = (uint64_t)(uintptr_t)dm;
  while (m) {
    const int src = (int)__builtin_ctzll(m);
    m &= m - 1;
    const uint64_t base = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(pd >> 32), src) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)pd, src);
    const int o0 = __builtin_amdgcn_readlane(T.o00, src), o1 = __builtin_amdgcn_readlane(T.o01, src);
    const int o2 = __builtin_amdgcn_readlane(T.o10, src), o3 = __builtin_amdgcn_readlane(T.o11, src);
    const float fa = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(T.fa), src));
    const float fb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(T.fb), src));
    const float g0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g[0]), src));
    const float g1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g[1]), src));
    const float g2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g[2]), src));
    if (lane < 12) {
      const int o = tap == 0 ? o0 : (tap == 1 ? o1 : (tap == 2 ? o2 : o3));
      const float wa = tap < 2 ? 1.f - fa : fa, wb = (tap & 1) ? fb : 1.f - fb;
      const float x = (c == 0 ? g0 : (c == 1 ? g1 : g2)) * (wa * wb);
      if (x != 0.f) {
        const long long q = __double2ll_rn((double)x * scale);
        atomicAdd(reinterpret_cast<unsigned long long*>((long long*)(uintptr_t)base + o + c), (unsigned long long)q);
      }
    }
  }
}

// The environment levels of one view as the shading adjoint sees them:
// texels, gradient maps, sizes and the float offset of the level's LDS copy
// (-1: not privatised).  Filled from wave-uniform values once per view; a lane
// picks its specular level (0..5) with selects rather than an indexed load.
struct LevelSet {
  const float* lvl[7];
  float* dlvl[7];
  long long* dfx[7];
  int lh[7], lw[7], off[7];
};
// (the empty asm keeps the compiler from folding the select chain back into
// an indexed load, which would put the level table in scratch memory)
template <class T>
__device__ __forceinline__ T pick_level(const T a[7], int l) {
  T r = a[0];
#pragma unroll
  for (int i = 1; i < 6; ++i) {
    r = l == i ? a[i] : r;
    asm volatile("" : "+v"(r));
  }
  return r;
}

// Adjoint of shade_forward for one record, in stages: every load of a record
// is issued before any of its atomics (a wave's memory counter retires in
// issue order, so a load issued after an atomic would wait for it).  (Keeping
// two records in flight, the loads of the next before the atomics of the
// current one, measured no faster and needs more registers.)
//   shade_load:    the record's 11 gradients and the surfel's parameters;
//   shade_fetch:   directions, taps, and the loads of the BRDF table and of
//                  the three environment lookups;
//   shade_adjoint: g = dL/dcol through the split-sum colour to dL/d(position,
//                  n_hat, albedo, roughness, metallic) and the texel gradients;
//   shade_scatter: the texel gradients into the levels and the 11 surfel
//                  gradients of the record into sg.
struct PPtrs { const float* p[7]; };

struct ShadeIn {
  long long r, s;  // record and surfel; r < 0: none
  float4 ga, gb, gc;  // the record's gradient slots 0..11
  float p[3], n[3], rho[3], rough, metal;
};
struct ShadeSt {
  long long r;  // < 0: no work (no record, or a record without gradient)
  float g[3], rho[3], rough, metal;
  float nh[3], wo[3], wl, nv, rd[3], tl, fx, fy;
  int l0;
  Tap Td, Ta, Tb;
  float lt[8], td[12], ta[12], tb[12];
};
struct ShadeOut {
  long long r;
  int l0;
  Tap Td, Ta, Tb;
  float gLd[3], gXa[3], gXb[3];
  float gp[3], gnh[3], grho[3], grough, gmetal;
};

__device__ inline void shade_load(const PPtrs& PP, long long N, const float* __restrict__ grad, long long r,
                                  long long s, ShadeIn& in) {
  in.r = r;
  in.s = s;
  if (r < 0) return;
  const float4* g4 = reinterpret_cast<const float4*>(grad + r * kGradStride);
  in.ga = g4[0];
  in.gb = g4[1];
  in.gc = g4[2];
  for (int k = 0; k < 3; ++k) {
    in.p[k] = PP.p[0][k * N + s];
    in.n[k] = PP.p[1][k * N + s];
    in.rho[k] = PP.p[4][k * N + s];
  }
  in.rough = PP.p[5][s];
  in.metal = PP.p[6][s];
}

__device__ inline void shade_fetch(const LevelSet& LS, const float cam_o[3], const Params& P, const ShadeIn& in,
                                   ShadeSt& S) {
  S.r = -1;
  if (in.r < 0) return;
  const float gr[11] = {in.ga.x, in.ga.y, in.ga.z, in.ga.w, in.gb.x, in.gb.y,
                        in.gb.z, in.gb.w, in.gc.x, in.gc.y, in.gc.z};
  bool any = false;
  for (int k = 0; k < kNGrad; ++k) any |= gr[k] != 0.f;
  // a record with a gradient was rasterised, hence kept by the cull
  if (!any) return;
  S.r = in.r;
  S.g[0] = gr[G_CR]; S.g[1] = gr[G_CG]; S.g[2] = gr[G_CB];
  for (int c = 0; c < 3; ++c) S.rho[c] = in.rho[c];
  S.rough = in.rough;
  S.metal = in.metal;
  const float nn = sqrtf(in.n[0] * in.n[0] + in.n[1] * in.n[1] + in.n[2] * in.n[2]);
  for (int c = 0; c < 3; ++c) S.nh[c] = in.n[c] / nn;
  const float wv[3] = {cam_o[0] - in.p[0], cam_o[1] - in.p[1], cam_o[2] - in.p[2]};
  S.wl = sqrtf(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
  const float iwl = 1.f / S.wl;
  for (int c = 0; c < 3; ++c) S.wo[c] = wv[c] * iwl;
  S.nv = S.nh[0] * S.wo[0] + S.nh[1] * S.wo[1] + S.nh[2] * S.wo[2];
  for (int c = 0; c < 3; ++c) S.rd[c] = 2.f * S.nv * S.nh[c] - S.wo[c];
  const float rc = clamp01(in.rough);
  const float lam = 5.f * rc;
  S.l0 = min((int)floorf(lam), 4);
  S.tl = lam - (float)S.l0;
  const int l1 = S.l0 + 1;
  // taps: irradiance level at n, the two specular levels at r_dir, BRDF table
  tap_setup(S.nh, LS.lh[6], LS.lw[6], S.Td);
  tap_setup(S.rd, pick_level(LS.lh, S.l0), pick_level(LS.lw, S.l0), S.Ta);
  tap_setup(S.rd, pick_level(LS.lh, l1), pick_level(LS.lw, l1), S.Tb);
  const float lx = clamp01(S.nv) * (float)(P.lut_nv - 1), ly = rc * (float)(P.lut_r - 1);
  const int j0 = min((int)floorf(lx), P.lut_nv - 2), i0 = min((int)floorf(ly), P.lut_r - 2);
  S.fx = lx - (float)j0;
  S.fy = ly - (float)i0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    S.lt[4 * c + 0] = P.lut[(i0 * P.lut_nv + j0) * 2 + c];
    S.lt[4 * c + 1] = P.lut[(i0 * P.lut_nv + j0 + 1) * 2 + c];
    S.lt[4 * c + 2] = P.lut[((i0 + 1) * P.lut_nv + j0) * 2 + c];
    S.lt[4 * c + 3] = P.lut[((i0 + 1) * P.lut_nv + j0 + 1) * 2 + c];
  }
  tap_fetch(LS.lvl[6], S.Td, S.td);
  tap_fetch(pick_level(LS.lvl, S.l0), S.Ta, S.ta);
  tap_fetch(pick_level(LS.lvl, l1), S.Tb, S.tb);
}

__device__ inline void shade_adjoint(const Params& P, const ShadeSt& S, ShadeOut& O) {
  O.r = S.r;
  O.l0 = 0;
  if (S.r < 0) return;
  O.l0 = S.l0;
  O.Td = S.Td;
  O.Ta = S.Ta;
  O.Tb = S.Tb;
  const float* g = S.g;
  const float* rho = S.rho;
  const float metal = S.metal, tl = S.tl, fx = S.fx, fy = S.fy, nv = S.nv;
  float beta[2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
    beta[c] = (1.f - fy) * ((1.f - fx) * S.lt[4 * c] + fx * S.lt[4 * c + 1]) +
              fy * ((1.f - fx) * S.lt[4 * c + 2] + fx * S.lt[4 * c + 3]);
  float F0[3], kd[3], gLs[3], gF0[3];
  for (int c = 0; c < 3; ++c) {
    F0[c] = 0.04f * (1.f - metal) + rho[c] * metal;
    kd[c] = (1.f - F0[c]) * (1.f - metal);
    gLs[c] = g[c] * (F0[c] * beta[0] + beta[1]);
    gF0[c] = 0.f;
    O.gLd[c] = g[c] * kd[c] * rho[c];
    O.gXa[c] = (1.f - tl) * gLs[c];
    O.gXb[c] = tl * gLs[c];
    O.gp[c] = 0.f;
    O.gnh[c] = 0.f;
    O.grho[c] = 0.f;
  }
  O.grough = 0.f;
  O.gmetal = 0.f;
  // diffuse: L_d(n)
  {
    float Ld[3];
    tap_adjoint(S.Td, S.td, S.nh, O.gLd, Ld, O.gnh);
    for (int c = 0; c < 3; ++c) {
      const float gkd = g[c] * rho[c] * Ld[c];
      O.grho[c] += g[c] * kd[c] * Ld[c];
      gF0[c] -= gkd * (1.f - metal);
      O.gmetal -= gkd * (1.f - F0[c]);
    }
  }
  // specular: the two levels around lambda, weights (1 - t) and t
  float gb1 = 0.f, gb2 = 0.f, gtl = 0.f, grd[3] = {0.f, 0.f, 0.f};
  {
    float A[3], B[3];
    tap_adjoint(S.Ta, S.ta, S.rd, O.gXa, A, grd);
    tap_adjoint(S.Tb, S.tb, S.rd, O.gXb, B, grd);
    for (int c = 0; c < 3; ++c) {
      const float Ls = (1.f - tl) * A[c] + tl * B[c];
      gF0[c] += g[c] * Ls * beta[0];
      gb1 += g[c] * Ls * F0[c];
      gb2 += g[c] * Ls;
      gtl += gLs[c] * (B[c] - A[c]);
    }
  }
  for (int c = 0; c < 3; ++c) {
    O.gmetal += gF0[c] * (rho[c] - 0.04f);
    O.grho[c] += gF0[c] * metal;
  }
  float g_rc = 5.f * gtl;
  // BRDF table slopes
  float gnvc = 0.f;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const float t00 = S.lt[4 * c], t01 = S.lt[4 * c + 1], t10 = S.lt[4 * c + 2], t11 = S.lt[4 * c + 3];
    const float dx = (1.f - fy) * (t01 - t00) + fy * (t11 - t10);
    const float dy = (1.f - fx) * (t10 - t00) + fx * (t11 - t01);
    const float gc = (c == 0) ? gb1 : gb2;
    gnvc += gc * dx * (float)(P.lut_nv - 1);
    g_rc += gc * dy * (float)(P.lut_r - 1);
  }
  float gnv = (nv >= 0.f && nv <= 1.f) ? gnvc : 0.f;
  const float nhg = S.nh[0] * grd[0] + S.nh[1] * grd[1] + S.nh[2] * grd[2];
  gnv += 2.f * nhg;
  float gwo[3];
  for (int i = 0; i < 3; ++i) {
    O.gnh[i] += 2.f * nv * grd[i] + gnv * S.wo[i];
    gwo[i] = -grd[i] + gnv * S.nh[i];
  }
  if (S.rough >= 0.f && S.rough <= 1.f) O.grough += g_rc;
  const float wg = S.wo[0] * gwo[0] + S.wo[1] * gwo[1] + S.wo[2] * gwo[2];
  const float iwl = 1.f / S.wl;
  for (int i = 0; i < 3; ++i) O.gp[i] -= (gwo[i] - S.wo[i] * wg) * iwl;
}

// Called by every lane of the wave (the global maps are written cooperatively);
// lanes without a record to scatter have O.r < 0.
template <bool DET>
__device__ inline void shade_scatter(const LevelSet& LS, const ShadeOut& O, float* sm, float* __restrict__ sg,
                                     double fx_scale) {
  const bool act = O.r >= 0;
  const int l1 = O.l0 + 1;
  const Tap* taps[3] = {&O.Td, &O.Ta, &O.Tb};
  const float* gs[3] = {O.gLd, O.gXa, O.gXb};
  if constexpr (DET) {
    long long* const gfx[3] = {LS.dfx[6], pick_level(LS.dfx, O.l0), pick_level(LS.dfx, l1)};
#pragma unroll
    for (int i = 0; i < 3; ++i) tap_scatter_global_wave_fx(act, gfx[i], *taps[i], gs[i], fx_scale);
  } else {
    const int offs[3] = {LS.off[6], pick_level(LS.off, O.l0), pick_level(LS.off, l1)};
    float* const gls[3] = {LS.dlvl[6], pick_level(LS.dlvl, O.l0), pick_level(LS.dlvl, l1)};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (act && offs[i] >= 0) tap_scatter_lds((lds_f32*)sm + offs[i], *taps[i], gs[i]);
      tap_scatter_global_wave(act && offs[i] < 0, gls[i], *taps[i], gs[i]);
    }
  }
  if (act) {
    float4* out = reinterpret_cast<float4*>(sg + O.r * 12);
    out[0] = make_float4(O.gp[0], O.gp[1], O.gp[2], O.gnh[0]);
    out[1] = make_float4(O.gnh[1], O.gnh[2], O.grho[0], O.grho[1]);
    out[2] = make_float4(O.grho[2], O.grough, O.gmetal, 0.f);
  }
}

// ---------------------------------------------------------------- raster params
// Projective form of the centre-precomputed MIP kernel from the centre Jacobian
// M = d(x,y)/d(u,v) and the depth slopes g = (t'_uz, t'_vz)/z:
//   K = M M^T, det A = det(M)^2, det B = det A + sigma tr K + sigma^2,
//   Q = (adj K + sigma I)/det B = (M M^T + sigma I)^{-1},
//   n_f = sqrt(det A / det B)                  (= sqrt(|I|/|Sigma_mip|), eq:mip_eval)
//   a3 = (g2 M21 - g1 M22)/det M,  b3 = (M12 g1 - M11 g2)/det M.
struct RasterGeo {
  float K11, K12, K22, trA, detB, Qxx, Qxy, Qyy, nf, a3, b3;
};
__device__ inline void raster_geometry(const Geo& o, float sigma, RasterGeo& r) {
  r.K11 = o.M11 * o.M11 + o.M12 * o.M12;
  r.K12 = o.M11 * o.M21 + o.M12 * o.M22;
  r.K22 = o.M21 * o.M21 + o.M22 * o.M22;
  r.trA = r.K11 + r.K22;
  r.detB = o.detA + sigma * r.trA + sigma * sigma;
  float ib = 1.f / r.detB;
  r.Qxx = (r.K22 + sigma) * ib;
  r.Qxy = -r.K12 * ib;
  r.Qyy = (r.K11 + sigma) * ib;
  r.nf = sqrtf(o.detA * ib);
  float idm = 1.f / o.dm;
  r.a3 = (o.g2 * o.M21 - o.g1 * o.M22) * idm;
  r.b3 = (o.M12 * o.g1 - o.M11 * o.g2) * idm;
}

// The raster parameters above evaluated in FP64 from the FP32 inputs and
// rounded once.  The projected centre is stored relative to the centre of the
// pixel rectangle's first pixel (its integer corner + 1/2, a few pixels at
// most), so the pixel offset d that the raster forms (one integer difference and
// one subtraction) is accurate to ~1e-7 px instead of the ~1e-4 px an FP32 centre
// near x = 1000 px would carry; thin (edge-on) ellipses amplify that error.
struct RasterGeoF {
  float x0r, y0r, Qxx, Qxy2, Qyy, a3, b3, nf;
};
__device__ inline void raster_geometry_f64(const float pf[3], const float nf_[3], const float tf[3],
                                           float su_, float sv_, const ViewDev& v, float sigma_,
                                           int il, int jl, RasterGeoF& out) {
  const double n0 = nf_[0], n1 = nf_[1], n2 = nf_[2];
  const double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  // one FP64 division per denominator, then products (each FP64 division is a
  // long instruction sequence; the results are rounded to FP32 once anyway)
  const double inn = 1.0 / nn;
  const double nh[3] = {n0 * inn, n1 * inn, n2 * inn};
  const double d = tf[0] * nh[0] + tf[1] * nh[1] + tf[2] * nh[2];
  double g[3] = {tf[0] - d * nh[0], tf[1] - d * nh[1], tf[2] - d * nh[2]};
  const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  const double ign = 1.0 / gn;
  const double uh[3] = {g[0] * ign, g[1] * ign, g[2] * ign};
  const double vh[3] = {nh[1] * uh[2] - nh[2] * uh[1], nh[2] * uh[0] - nh[0] * uh[2],
                        nh[0] * uh[1] - nh[1] * uh[0]};
  const double su = su_, sv = sv_, sigma = sigma_;
  double cp[3], up[3], vp[3];
  for (int i = 0; i < 3; ++i) {
    const float* R = v.R + 3 * i;
    cp[i] = (double)R[0] * pf[0] + (double)R[1] * pf[1] + (double)R[2] * pf[2] + (double)v.t[i];
    up[i] = su * ((double)R[0] * uh[0] + (double)R[1] * uh[1] + (double)R[2] * uh[2]);
    vp[i] = sv * ((double)R[0] * vh[0] + (double)R[1] * vh[1] + (double)R[2] * vh[2]);
  }
  const double z = cp[2], iz = 1.0 / z, mx = cp[0] * iz, my = cp[1] * iz;
  const double fx = v.fx, fy = v.fy;
  const double x0 = fx * mx + (double)v.cx, y0 = fy * my + (double)v.cy;
  const double M11 = fx * (up[0] - mx * up[2]) * iz, M12 = fx * (vp[0] - mx * vp[2]) * iz;
  const double M21 = fy * (up[1] - my * up[2]) * iz, M22 = fy * (vp[1] - my * vp[2]) * iz;
  const double g1 = up[2] * iz, g2 = vp[2] * iz;
  const double dm = M11 * M22 - M12 * M21;
  const double detA = dm * dm;
  const double K11 = M11 * M11 + M12 * M12, K12 = M11 * M21 + M12 * M22, K22 = M21 * M21 + M22 * M22;
  const double detB = detA + sigma * (K11 + K22) + sigma * sigma;
  // the centre relative to the first pixel centre of the rectangle, rounded once
  out.x0r = (float)(x0 - ((double)il + 0.5));
  out.y0r = (float)(y0 - ((double)jl + 0.5));
  const double ib = 1.0 / detB, idm = 1.0 / dm;
  out.Qxx = (float)((K22 + sigma) * ib);
  out.Qxy2 = (float)(-2.0 * K12 * ib);
  out.Qyy = (float)((K11 + sigma) * ib);
  out.nf = (float)sqrt(detA * ib);
  out.a3 = (float)((g2 * M21 - g1 * M22) * idm);
  out.b3 = (float)((M12 * g1 - M11 * g2) * idm);
}

__device__ inline void load_surfel(const float* const* P, long long N, long long s, float p[3],
                                   float n[3], float t[3], float& su, float& sv) {
  for (int k = 0; k < 3; ++k) {
    p[k] = P[0][k * N + s];
    n[k] = P[1][k * N + s];
    t[k] = P[2][k * N + s];
  }
  su = P[3][s];
  sv = P[3][N + s];
}

__global__ void __launch_bounds__(256) preprocess_kernel(PPtrs PP, long long N, const ViewDev* __restrict__ views,
                                                         int v0, Params prm, float* __restrict__ recs,
                                                         uint32_t* __restrict__ counts,
                                                         uint32_t* __restrict__ zkey, uint2* __restrict__ prect) {
  const int vi = v0 + blockIdx.y;
  const ViewDev& v = views[vi];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.n_surf) return;
  const long long s = v.surf_off + i;
  const long long r = v.rec_off + i;
  float p[3], n[3], t[3], su, sv;
  load_surfel(PP.p, N, s, p, n, t, su, sv);
  Geo o;
  bin_geometry(p, n, t, su, sv, v, prm.r_cut, prm.sigma_f, o);
  float4* out = reinterpret_cast<float4*>(recs + r * kRecFloats);
  if (!o.keep) {
    counts[r] = 0u;
    zkey[r] = 0xffffffffu;
    prect[r] = make_uint2(1u, 0u);
    float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    out[0] = z4; out[1] = z4; out[2] = z4;
    out[3] = make_float4(__int_as_float(1), __int_as_float(0), __int_as_float(0xffffffff), 0.f);
    return;
  }
  RasterGeoF g;
  raster_geometry_f64(p, n, t, su, sv, v, prm.sigma_f, o.il, o.jl, g);
  float col[3];
  if (prm.shade == 0) {
    for (int c = 0; c < 3; ++c) col[c] = PP.p[4][c * N + s];
  } else if (prm.shade == 2) {
    for (int c = 0; c < 3; ++c) col[c] = o.nh[c];
  } else {
    float rho[3] = {PP.p[4][s], PP.p[4][N + s], PP.p[4][2 * N + s]};
    shade_forward(v, prm, p, o.nh, rho, PP.p[5][s], PP.p[6][s], col);
  }
  const int tw = prm.tile_w, th = prm.tile_h;
  const int tx0 = o.il / tw, tx1 = o.ih / tw, ty0 = o.jl / th, ty1 = o.jh / th;
  counts[r] = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
  zkey[r] = __float_as_uint(o.zs);
  prect[r] = make_uint2((uint32_t)(o.il | (o.ih << 16)), (uint32_t)(o.jl | (o.jh << 16)));
  out[0] = make_float4(g.x0r, g.y0r, g.Qxx, g.Qxy2);
  out[1] = make_float4(g.Qyy, g.a3, g.b3, g.nf);
  out[2] = make_float4(o.ze, col[0], col[1], col[2]);
  out[3] = make_float4(__int_as_float(o.il | (o.ih << 16)), __int_as_float(o.jl | (o.jh << 16)),
                       o.zs, __uint_as_float((uint32_t)r));
}

hipError_t launch_preprocess(const float* const P[7], long long N, const ViewDev* views, int v0,
                             int v1, int max_surf, const Params& prm, float* recs,
                             uint32_t* counts, uint32_t* zkey, uint2* prect, hipStream_t st) {
  if (v1 <= v0 || max_surf <= 0) return hipSuccess;
  PPtrs PP;
  for (int k = 0; k < 7; ++k) PP.p[k] = P[k];
  dim3 grid((max_surf + 255) / 256, v1 - v0);
  hipLaunchKernelGGL(preprocess_kernel, grid, dim3(256), 0, st, PP, N, views, v0, prm, recs, counts, zkey,
                     prect);
  return hipGetLastError();
}

// ---------------------------------------------------------------- backward
struct GPtrs { float* p[7]; };

// Surfel adjoint in two kernels.
//   shade_backward_kernel (split-sum only): one thread per record, striding over
//   the records of one scene view by view.  The adjoint of the split-sum colour gives
//   dL/d(position, n_hat, albedo, roughness, metallic) of that record (written
//   to sg[r][12]) and the texel gradients of the environment levels: the small
//   levels accumulate in a block-private LDS copy (written out as a per-block
//   partial and summed in a fixed order by envmap_partial_reduce*), the large
//   ones take global atomics.
//   geometry_backward_kernel: one thread per surfel; for every view of its
//   scene it reads the 11 record gradients (and sg), applies the adjoint of
//   bin_geometry / raster_geometry and sums over views in registers, so the
//   parameter gradients are written once and deterministically.  On request
//   it also sums the screen-space statistic (slot G_SS) over the views and
//   counts the views whose record survived the cull (non-empty rectangle).
struct LocalMaps {
  int off[7];  // float offset of level l in the LDS copy, -1 if not privatised
  int total;   // floats
};
struct SceneViews {
  int idx[kMaxViews];
  int n;
  int n_surf;
  long long surf_off;
};

__device__ inline bool record_has_grad(const float* grad, long long r, float gr[12]) {
  const float4* g4 = reinterpret_cast<const float4*>(grad + r * kGradStride);
  const float4 a = g4[0], b = g4[1], c = g4[2];
  gr[0] = a.x; gr[1] = a.y; gr[2] = a.z; gr[3] = a.w;
  gr[4] = b.x; gr[5] = b.y; gr[6] = b.z; gr[7] = b.w;
  gr[8] = c.x; gr[9] = c.y; gr[10] = c.z; gr[11] = 0.f;
  bool any = false;
  for (int k = 0; k < kNGrad; ++k) any |= gr[k] != 0.f;
  return any;
}

template <bool DET>
__global__ void __launch_bounds__(kBackwardThreads, 1) shade_backward_kernel(
    PPtrs PP, long long N, const ViewDev* __restrict__ views, SceneViews sv, Params prm,
    const float* __restrict__ grad, float* __restrict__ sg, LocalMaps lm, float* __restrict__ partial,
    const int* __restrict__ fx_exp) {
  extern __shared__ float sm[];
  const double fx_scale = DET ? ldexp(1.0, *fx_exp) : 0.0;
  for (int i = threadIdx.x; i < lm.total; i += blockDim.x) sm[i] = 0.f;
  __syncthreads();
  const long long stride = (long long)gridDim.x * blockDim.x;
  // a wave's lanes take consecutive records; the loop runs while the wave's
  // first lane has a record, so every lane stays in it (the scatter into the
  // global maps needs the whole wave)
  const long long wave0 = (long long)blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
  const long long first = wave0 + (threadIdx.x & 63);
  // the view loop is uniform, so the view's descriptor stays in scalar registers
  for (int k = 0; k < sv.n; ++k) {
    const ViewDev& v = views[sv.idx[k]];
    LevelSet LS;
#pragma unroll
    for (int l = 0; l < 7; ++l) {
      LS.lvl[l] = v.lvl[l];
      LS.dlvl[l] = v.dlvl[l];
      LS.dfx[l] = v.dlvl_fx[l];
      LS.lh[l] = v.lh[l];
      LS.lw[l] = v.lw[l];
      LS.off[l] = lm.off[l];
    }
    const float cam_o[3] = {v.cam_o[0], v.cam_o[1], v.cam_o[2]};
    const long long rec_off = v.rec_off, n = sv.n_surf;
    auto rec = [&](long long local) { return local < n ? rec_off + local : -1ll; };
    for (long long w = wave0, local = first; w < n; w += stride, local += stride) {
      ShadeIn in;
      ShadeSt S;
      ShadeOut O;
      shade_load(PP, N, grad, rec(local), sv.surf_off + local, in);
      shade_fetch(LS, cam_o, prm, in, S);
      shade_adjoint(prm, S, O);
      shade_scatter<DET>(LS, O, sm, sg, fx_scale);
    }
  }
  if (lm.total > 0) {
    __syncthreads();
    float* dstp = partial + (long long)blockIdx.x * lm.total;
    for (int i = threadIdx.x; i < lm.total; i += blockDim.x) dstp[i] = sm[i];
  }
}

__global__ void __launch_bounds__(256) geometry_backward_kernel(
    PPtrs PP, long long N, const ViewDev* __restrict__ views, int n_views, Params prm,
    const float* __restrict__ grad, const float* __restrict__ sg, GPtrs G,
    const float* __restrict__ recs, float* __restrict__ ss_out, int* __restrict__ vis_out,
    const int* __restrict__ status) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  float p[3], n[3], t[3], su, sv;
  load_surfel(PP.p, N, s, p, n, t, su, sv);
  float gp[3] = {0, 0, 0}, gn[3] = {0, 0, 0}, gt[3] = {0, 0, 0}, gsu = 0.f, gsv = 0.f;
  float grho[3] = {0, 0, 0}, grough = 0.f, gmetal = 0.f;
  float ss_sum = 0.f;
  int n_vis = 0;
  const float sig = prm.sigma_f;
  for (int vi = 0; vi < n_views; ++vi) {
    const ViewDev& v = views[vi];
    if (s < v.surf_off || s >= v.surf_off + v.n_surf) continue;
    const long long r = v.rec_off + (s - v.surf_off);
    if (ss_out) ss_sum += grad[r * kGradStride + G_SS];
    if (vis_out) {
      // culled records carry the empty rectangle i_lo = 1 > i_hi = 0
      const uint32_t rx = __float_as_uint(recs[r * kRecFloats + R_RX]);
      n_vis += (rx & 0xffffu) <= (rx >> 16) ? 1 : 0;
    }
    float gr[12];
    // depth-consolidation term: gradient with respect to T4z = c'_z
    const float gtz = prm.cons ? grad[r * kGradStride + G_TZ] : 0.f;
    const bool has = record_has_grad(grad, r, gr);
    if (!has && gtz == 0.f) continue;
    Geo o;
    bin_geometry(p, n, t, su, sv, v, prm.r_cut, sig, o);
    if (!o.keep) continue;
    RasterGeo g;
    raster_geometry(o, sig, g);
    float gnh[3] = {0, 0, 0};
    // colour
    if (prm.shade == 0) {
      grho[0] += gr[G_CR]; grho[1] += gr[G_CG]; grho[2] += gr[G_CB];
    } else if (prm.shade == 2) {
      gnh[0] += gr[G_CR]; gnh[1] += gr[G_CG]; gnh[2] += gr[G_CB];
    } else if (has) {
      // sg holds the shading adjoint of the records with a gradient (the others
      // have dL/dcol = 0)
      const float4* in = reinterpret_cast<const float4*>(sg + r * 12);
      const float4 a = in[0], b = in[1], c = in[2];
      gp[0] += a.x; gp[1] += a.y; gp[2] += a.z;
      gnh[0] += a.w; gnh[1] += b.x; gnh[2] += b.y;
      grho[0] += b.z; grho[1] += b.w; grho[2] += c.x;
      grough += c.y; gmetal += c.z;
    }
    // MIP kernel parameters -> M, g
    const float detB = g.detB, dm = o.dm;
    const float gQxx = gr[G_QXX], gQxy = 2.f * gr[G_QXY2], gQyy = gr[G_QYY];
    const float gnf = gr[G_NF], ga3 = gr[G_A3], gb3 = gr[G_B3];
    const float ib = 1.f / detB;  // one reciprocal per denominator, then products
    float gdetB = -(gQxx * g.Qxx + gQxy * g.Qxy + gQyy * g.Qyy) * ib;
    float gdetA = 0.f;
    if (g.nf > 0.f) {
      gdetB += -gnf * g.nf * (0.5f * ib);
      gdetA += gnf * (0.5f * ib) / g.nf;
    }
    float gK22 = gQxx * ib, gK12 = -gQxy * ib, gK11 = gQyy * ib;
    gdetA += gdetB;
    const float gtrA = sig * gdetB;
    gK11 += gtrA;
    gK22 += gtrA;
    float gdm = 2.f * dm * gdetA;
    float gM11 = 0.f, gM12 = 0.f, gM21 = 0.f, gM22 = 0.f, gg1 = 0.f, gg2 = 0.f;
    const float idm = 1.f / dm;
    gg2 += ga3 * o.M21 * idm; gM21 += ga3 * o.g2 * idm;
    gg1 -= ga3 * o.M22 * idm; gM22 -= ga3 * o.g1 * idm;
    gdm -= ga3 * g.a3 * idm;
    gM12 += gb3 * o.g1 * idm; gg1 += gb3 * o.M12 * idm;
    gM11 -= gb3 * o.g2 * idm; gg2 -= gb3 * o.M11 * idm;
    gdm -= gb3 * g.b3 * idm;
    gM11 += 2.f * o.M11 * gK11 + o.M21 * gK12;
    gM12 += 2.f * o.M12 * gK11 + o.M22 * gK12;
    gM21 += 2.f * o.M21 * gK22 + o.M11 * gK12;
    gM22 += 2.f * o.M22 * gK22 + o.M12 * gK12;
    gM11 += o.M22 * gdm; gM22 += o.M11 * gdm;
    gM12 -= o.M21 * gdm; gM21 -= o.M12 * gdm;
    // M, g, x0, y0 -> camera-space c', t'_u, t'_v
    const float z = o.z, iz = 1.f / z, fx = v.fx, fy = v.fy;
    float gcp[3] = {0, 0, 0}, gup[3] = {0, 0, 0}, gvp[3] = {0, 0, 0};
    float gmx = fx * gr[G_X0], gmy = fy * gr[G_Y0], gz = gtz;
    gup[0] += fx * gM11 * iz; gup[2] -= fx * o.mx * gM11 * iz; gmx -= fx * o.up[2] * gM11 * iz; gz -= o.M11 * gM11 * iz;
    gvp[0] += fx * gM12 * iz; gvp[2] -= fx * o.mx * gM12 * iz; gmx -= fx * o.vp[2] * gM12 * iz; gz -= o.M12 * gM12 * iz;
    gup[1] += fy * gM21 * iz; gup[2] -= fy * o.my * gM21 * iz; gmy -= fy * o.up[2] * gM21 * iz; gz -= o.M21 * gM21 * iz;
    gvp[1] += fy * gM22 * iz; gvp[2] -= fy * o.my * gM22 * iz; gmy -= fy * o.vp[2] * gM22 * iz; gz -= o.M22 * gM22 * iz;
    gup[2] += gg1 * iz; gz -= o.g1 * gg1 * iz;
    gvp[2] += gg2 * iz; gz -= o.g2 * gg2 * iz;
    gcp[0] += gmx * iz; gz -= o.mx * gmx * iz;
    gcp[1] += gmy * iz; gz -= o.my * gmy * iz;
    gcp[2] += gz;
    // rotate back to world space: g_world = R^T g_cam
    float gtu[3], gtv[3];
    for (int j = 0; j < 3; ++j) {
      gp[j] += v.R[j] * gcp[0] + v.R[3 + j] * gcp[1] + v.R[6 + j] * gcp[2];
      gtu[j] = v.R[j] * gup[0] + v.R[3 + j] * gup[1] + v.R[6 + j] * gup[2];
      gtv[j] = v.R[j] * gvp[0] + v.R[3 + j] * gvp[1] + v.R[6 + j] * gvp[2];
    }
    // t_u = s_u u_hat, t_v = s_v v_hat
    gsu += o.uh[0] * gtu[0] + o.uh[1] * gtu[1] + o.uh[2] * gtu[2];
    gsv += o.vh[0] * gtv[0] + o.vh[1] * gtv[1] + o.vh[2] * gtv[2];
    float guh[3], gvh[3];
    for (int j = 0; j < 3; ++j) { guh[j] = su * gtu[j]; gvh[j] = sv * gtv[j]; }
    // v_hat = n_hat x u_hat
    gnh[0] += o.uh[1] * gvh[2] - o.uh[2] * gvh[1];
    gnh[1] += o.uh[2] * gvh[0] - o.uh[0] * gvh[2];
    gnh[2] += o.uh[0] * gvh[1] - o.uh[1] * gvh[0];
    guh[0] += gvh[1] * o.nh[2] - gvh[2] * o.nh[1];
    guh[1] += gvh[2] * o.nh[0] - gvh[0] * o.nh[2];
    guh[2] += gvh[0] * o.nh[1] - gvh[1] * o.nh[0];
    // u_hat = g / |g|
    float ug = o.uh[0] * guh[0] + o.uh[1] * guh[1] + o.uh[2] * guh[2];
    float gg[3];
    const float ign = 1.f / o.gn;
    for (int j = 0; j < 3; ++j) gg[j] = (guh[j] - o.uh[j] * ug) * ign;
    // g = t - (t.n_hat) n_hat
    float ngg = o.nh[0] * gg[0] + o.nh[1] * gg[1] + o.nh[2] * gg[2];
    for (int j = 0; j < 3; ++j) {
      gt[j] += gg[j] - ngg * o.nh[j];
      gnh[j] += -o.d * gg[j] - ngg * t[j];
    }
    // n_hat = n / |n|
    float ng = o.nh[0] * gnh[0] + o.nh[1] * gnh[1] + o.nh[2] * gnh[2];
    const float inn = 1.f / o.nn;
    for (int j = 0; j < 3; ++j) gn[j] += (gnh[j] - o.nh[j] * ng) * inn;
  }
  if (status && *status == 3 /* SS_ERR_CAPACITY: the forward's pair list was cut */) {
    const float q = __builtin_nanf("");
    for (int k = 0; k < 3; ++k) { gp[k] = gn[k] = gt[k] = grho[k] = q; }
    gsu = gsv = grough = gmetal = ss_sum = q;
  }
  if (ss_out) ss_out[s] = ss_sum;
  if (vis_out) vis_out[s] = n_vis;
  for (int k = 0; k < 3; ++k) {
    if (G.p[0]) G.p[0][k * N + s] = gp[k];
    if (G.p[1]) G.p[1][k * N + s] = gn[k];
    if (G.p[2]) G.p[2][k * N + s] = gt[k];
    if (G.p[4]) G.p[4][k * N + s] = grho[k];
  }
  if (G.p[3]) { G.p[3][s] = gsu; G.p[3][N + s] = gsv; }
  if (G.p[5]) G.p[5][s] = grough;
  if (G.p[6]) G.p[6][s] = gmetal;
}

struct LevelPtrs { float* p[7]; };

// Sums the per-block partials of the privatised levels in a fixed order, in two
// stages: kReduceSplit chunks of blocks, then the chunks, into the level
// gradients.
__global__ void envmap_partial_reduce1(const float* __restrict__ partial, int n_blocks, int total,
                                       float* __restrict__ stage) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int per = (n_blocks + kReduceSplit - 1) / kReduceSplit;
  const int b0 = blockIdx.y * per, b1 = min(b0 + per, n_blocks);
  float acc = 0.f;
  for (int b = b0; b < b1; ++b) acc += partial[(long long)b * total + i];
  stage[(long long)blockIdx.y * total + i] = acc;
}
__global__ void envmap_partial_reduce2(const float* __restrict__ stage, LocalMaps lm, LevelPtrs dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= lm.total) return;
  float acc = 0.f;
  for (int c = 0; c < kReduceSplit; ++c) acc += stage[(long long)c * lm.total + i];
  int l = -1, best = -1;
  for (int k = 0; k < 7; ++k)
    if (lm.off[k] >= 0 && lm.off[k] <= i && lm.off[k] > best) { best = lm.off[k]; l = k; }
  dst.p[l][i - best] = acc;
}

int backward_blocks(long long n_items) {
  long long b = (n_items + kBackwardThreads - 1) / kBackwardThreads;
  return (int)(b < kBackwardBlocks ? (b > 0 ? b : 1) : kBackwardBlocks);
}

hipError_t launch_shade_backward(const float* const P[7], long long N, const ViewDev* views,
                                 const int* scene_views, int n_scene_views, long long surf_off,
                                 int n_surf, const int local_off[7], int local_total, float* partial,
                                 float* const level_grad[7], const Params& prm, const float* grad,
                                 float* sg, const int* fx_exp, hipStream_t st) {
  if (n_surf <= 0 || n_scene_views <= 0) return hipSuccess;
  if (fx_exp && local_total != 0) return hipErrorInvalidValue;
  PPtrs PP;
  for (int k = 0; k < 7; ++k) PP.p[k] = P[k];
  SceneViews sv;
  for (int k = 0; k < n_scene_views; ++k) sv.idx[k] = scene_views[k];
  sv.n = n_scene_views;
  sv.n_surf = n_surf;
  sv.surf_off = surf_off;
  LocalMaps lm;
  lm.total = local_total;
  for (int l = 0; l < 7; ++l) lm.off[l] = local_total > 0 ? local_off[l] : -1;
  const int nb = backward_blocks((long long)n_surf * n_scene_views);
  if (fx_exp) {
    hipLaunchKernelGGL(shade_backward_kernel<true>, dim3(nb), dim3(kBackwardThreads), 0, st, PP, N, views, sv,
                       prm, grad, sg, lm, partial, fx_exp);
    return hipGetLastError();
  }
  static bool lds_attr = false;  // allow the privatised levels beyond the default dynamic-LDS limit
  if (!lds_attr) {
    hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(&shade_backward_kernel<false>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        kLocalMapFloats * (int)sizeof(float));
    if (ea != hipSuccess) return ea;
    lds_attr = true;
  }
  hipLaunchKernelGGL(shade_backward_kernel<false>, dim3(nb), dim3(kBackwardThreads),
                     (size_t)local_total * sizeof(float), st, PP, N, views, sv, prm, grad, sg, lm,
                     partial, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || local_total == 0) return e;
  LevelPtrs lp;
  for (int l = 0; l < 7; ++l) lp.p[l] = level_grad[l];
  float* stage = partial + (long long)kBackwardBlocks * kLocalMapFloats;
  hipLaunchKernelGGL(envmap_partial_reduce1, dim3((local_total + 255) / 256, kReduceSplit), dim3(256), 0,
                     st, partial, nb, local_total, stage);
  hipLaunchKernelGGL(envmap_partial_reduce2, dim3((local_total + 255) / 256), dim3(256), 0, st, stage,
                     lm, lp);
  return hipGetLastError();
}

hipError_t launch_geometry_backward(const float* const P[7], long long N, const ViewDev* views,
                                    int n_views, const Params& prm, const float* grad,
                                    const float* sg, float* const G[7], const float* recs,
                                    float* ss_out, int* vis_out, const int* status, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  PPtrs PP;
  GPtrs GG;
  for (int k = 0; k < 7; ++k) { PP.p[k] = P[k]; GG.p[k] = G[k]; }
  hipLaunchKernelGGL(geometry_backward_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, PP, N,
                     views, n_views, prm, grad, sg, GG, recs, ss_out, vis_out, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------- deterministic mode
// Per record the bound 2 max_c |dL/dc_c| max(1, max_c |albedo_c|) of its texel
// gradients, maxed into *bound as float bits (non-negative floats order like
// their bit patterns).
__global__ void fixed_point_bound_kernel(const float* __restrict__ grad, const float* __restrict__ albedo,
                                         long long N, const ViewDev* __restrict__ views, SceneViews sv,
                                         unsigned* __restrict__ bound) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float b = 0.f;
  if (i < sv.n_surf * sv.n) {
    const int k = (int)(i / sv.n_surf);
    const long long local = i - (long long)k * sv.n_surf;
    const ViewDev& v = views[sv.idx[k]];
    const long long r = v.rec_off + local, s = v.surf_off + local;
    const float4 g = reinterpret_cast<const float4*>(grad + r * kGradStride)[2];  // slots 8..11: CR, CG, CB, SS
    const float gc = fmaxf(fabsf(g.x), fmaxf(fabsf(g.y), fabsf(g.z)));
    const float ra = fmaxf(1.f, fmaxf(fabsf(albedo[s]), fmaxf(fabsf(albedo[N + s]), fabsf(albedo[2 * N + s]))));
    b = 2.f * gc * ra;
  }
  // a wave maximum, one atomic per wave
  for (int off = 32; off > 0; off >>= 1) b = fmaxf(b, __shfl_xor(b, off));
  if ((threadIdx.x & 63) == 0 && b > 0.f) atomicMax(bound, __float_as_uint(b));
}
__global__ void fixed_point_exponent_kernel(const unsigned* __restrict__ bound, long long n_rec, int* fx_exp) {
  const float b = __uint_as_float(*bound);
  int e = 0;
  // 36 n b < 2^61: s = 61 - ceil(log2(36 n b)); no contribution at all: any s
  const double t = 36.0 * (double)(n_rec > 0 ? n_rec : 1) * (double)b;
  if (t > 0.0 && t < 1e300) {
    (void)frexp(t, &e);  // t < 2^e
    *fx_exp = 61 - e;
  } else {
    *fx_exp = 0;
  }
}
hipError_t launch_fixed_point_scale(const float* grad, const float* albedo, long long N, const ViewDev* views,
                                    const int* scene_views, int n_scene_views, long long n_surf,
                                    unsigned* bound, int* fx_exp, hipStream_t st) {
  SceneViews sv;
  for (int k = 0; k < n_scene_views; ++k) sv.idx[k] = scene_views[k];
  sv.n = n_scene_views;
  sv.n_surf = (int)n_surf;
  sv.surf_off = 0;  // unused: each record's surfel comes from its view
  hipError_t e = launch_fill_u32(bound, 0u, 1, st);
  if (e != hipSuccess) return e;
  const long long n = n_surf * n_scene_views;
  if (n > 0)
    hipLaunchKernelGGL(fixed_point_bound_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, grad,
                       albedo, N, views, sv, bound);
  hipLaunchKernelGGL(fixed_point_exponent_kernel, dim3(1), dim3(1), 0, st, bound, n, fx_exp);
  return hipGetLastError();
}
__global__ void fixed_to_float_kernel(const long long* __restrict__ src, long long n, const int* __restrict__ fx_exp,
                                      float* __restrict__ dst) {
  const double inv = ldexp(1.0, -*fx_exp);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = (float)((double)src[i] * inv);
}
hipError_t launch_fixed_to_float(const long long* src, long long n, const int* fx_exp, float* dst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long b = (n + 255) / 256;
  hipLaunchKernelGGL(fixed_to_float_kernel, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, st, src, n,
                     fx_exp, dst);
  return hipGetLastError();
}

}  // namespace ss
