// Per (surfel, view) preprocessing and forward shading, and their adjoint.
//
// Forward (one thread per record): the binning decision (cull, depth interval,
// pixel rectangle; Sec. 3.1, Sec. 3.2.1, App. A.1), the centre-precomputed MIP
// kernel (Sec. 3.3.2) in projective form, and the split-sum colour (eq:ibl).
// Backward (one thread per surfel, looping over the views of its scene): the
// chain rule from the 11 record gradients written by the raster backward to
// position, normal, tangent, scale, albedo, roughness and metallic, plus texel
// gradients of the environment levels (atomics into small maps).
#include "common.h"

namespace ss {

// Address-space-qualified views of the environment levels: the level pointers
// come from the view descriptors at run time, so without the qualifier every
// texel load and gradient atomic would be a FLAT instruction (and atomics into
// the LDS-privatised levels would take the FLAT path instead of ds_add_f32).
typedef const __attribute__((address_space(1))) float gmem_cf32;
typedef __attribute__((address_space(1))) float gmem_f32;
typedef __attribute__((address_space(3))) float lds_f32;

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
  float a = th * ((float)H / kPi) - 0.5f;
  float b = ph * ((float)W / (2.f * kPi)) - 0.5f;
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
  float wo[3] = {wv[0] / wl, wv[1] / wl, wv[2] / wl};
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

// One bilinear lat-long lookup with its adjoint: returns the value, scatters
// g (the gradient of the looked-up value, known up front) into the texels of
// dm (LDS or global) and adds the gradient with respect to the direction d to gd.
template <class DST>
__device__ inline void latlong_lookup_adjoint(const float* mp, DST* dm, int H, int W, const float d[3],
                                              const float g[3], float val[3], float gd[3]) {
  gmem_cf32* m = (gmem_cf32*)mp;
  LatLong L;
  latlong_coords(d, H, W, L);
  const int o00 = 3 * (L.r0 * W + L.c0), o01 = 3 * (L.r0 * W + L.c1);
  const int o10 = 3 * (L.r1 * W + L.c0), o11 = 3 * (L.r1 * W + L.c1);
  const float w00 = (1.f - L.fa) * (1.f - L.fb), w01 = (1.f - L.fa) * L.fb;
  const float w10 = L.fa * (1.f - L.fb), w11 = L.fa * L.fb;
  float ga = 0.f, gb = 0.f;
  for (int c = 0; c < 3; ++c) {
    const float v00 = m[o00 + c], v01 = m[o01 + c], v10 = m[o10 + c], v11 = m[o11 + c];
    val[c] = w00 * v00 + w01 * v01 + w10 * v10 + w11 * v11;
    ga += g[c] * ((1.f - L.fb) * (v10 - v00) + L.fb * (v11 - v01));
    gb += g[c] * ((1.f - L.fa) * (v01 - v00) + L.fa * (v11 - v10));
    if (g[c] != 0.f) {
      grad_add(dm + o00 + c, g[c] * w00);
      grad_add(dm + o01 + c, g[c] * w01);
      grad_add(dm + o10 + c, g[c] * w10);
      grad_add(dm + o11 + c, g[c] * w11);
    }
  }
  const float gth = ga * ((float)H / kPi);
  const float gph = gb * ((float)W / (2.f * kPi));
  if (L.rho > 1e-20f && L.den > 0.f) {
    // th = atan2(rho, z), ph = atan2(y, x), rho = sqrt(x^2 + y^2)
    const float dth_drho = d[2] / L.den, dth_dz = -L.rho / L.den;
    const float r2 = L.rho * L.rho;
    gd[0] += gth * dth_drho * d[0] / L.rho - gph * d[1] / r2;
    gd[1] += gth * dth_drho * d[1] / L.rho + gph * d[0] / r2;
    gd[2] += gth * dth_dz;
  }
}

// Adjoint of shade_forward: given g = dL/dcol, accumulates into g_p, g_nh,
// g_rho, g_rough, g_metal and scatters texel gradients into level l's LDS
// copy (loc_off[l] >= 0) or its global gradient map.  Each lookup's adjoint
// needs only quantities known before the lookup, so the three lookups are
// processed one after the other (few live registers).
__device__ inline void level_lookup_adjoint(const ViewDev& v, const float* sm, const int loc_off[7], int l,
                                            const float d[3], const float g[3], float val[3], float gd[3]) {
  if (loc_off[l] >= 0)
    latlong_lookup_adjoint(v.lvl[l], (lds_f32*)sm + loc_off[l], v.lh[l], v.lw[l], d, g, val, gd);
  else
    latlong_lookup_adjoint(v.lvl[l], (gmem_f32*)v.dlvl[l], v.lh[l], v.lw[l], d, g, val, gd);
}

__device__ inline void shade_backward(const ViewDev& v, const Params& P, const float p[3],
                                      const float nh[3], const float rho[3], float rough,
                                      float metal, const float g[3], const float* sm,
                                      const int loc_off[7], float g_p[3], float g_nh[3],
                                      float g_rho[3], float& g_rough, float& g_metal) {
  float wv[3] = {v.cam_o[0] - p[0], v.cam_o[1] - p[1], v.cam_o[2] - p[2]};
  const float wl = sqrtf(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
  const float wo[3] = {wv[0] / wl, wv[1] / wl, wv[2] / wl};
  const float nv = nh[0] * wo[0] + nh[1] * wo[1] + nh[2] * wo[2];
  const float rd[3] = {2.f * nv * nh[0] - wo[0], 2.f * nv * nh[1] - wo[1], 2.f * nv * nh[2] - wo[2]};
  const float rc = clamp01(rough);
  const float lam = 5.f * rc;
  const int l0 = min((int)floorf(lam), 4);
  const float tl = lam - (float)l0;
  const float nvc = clamp01(nv);
  LutTap T;
  float beta[2];
  lut_fetch(P, nvc, rc, T, beta);
  float F0[3], kd[3], gLs[3], gF0[3];
  for (int c = 0; c < 3; ++c) {
    F0[c] = 0.04f * (1.f - metal) + rho[c] * metal;
    kd[c] = (1.f - F0[c]) * (1.f - metal);
    gLs[c] = g[c] * (F0[c] * beta[0] + beta[1]);
    gF0[c] = 0.f;
  }
  float gb1 = 0.f, gb2 = 0.f, gtl = 0.f, grd[3] = {0.f, 0.f, 0.f};
  // diffuse: L_d(n)
  {
    float gLd[3], Ld[3];
    for (int c = 0; c < 3; ++c) gLd[c] = g[c] * kd[c] * rho[c];
    level_lookup_adjoint(v, sm, loc_off, 6, nh, gLd, Ld, g_nh);
    for (int c = 0; c < 3; ++c) {
      const float gkd = g[c] * rho[c] * Ld[c];
      g_rho[c] += g[c] * kd[c] * Ld[c];
      gF0[c] -= gkd * (1.f - metal);
      g_metal -= gkd * (1.f - F0[c]);
    }
  }
  // specular: the two levels around lambda, weights (1 - t) and t
  for (int side = 0; side < 2; ++side) {
    const int l = l0 + side;
    const float wt = side ? tl : 1.f - tl;
    float gX[3], X[3];
    for (int c = 0; c < 3; ++c) gX[c] = wt * gLs[c];
    level_lookup_adjoint(v, sm, loc_off, l, rd, gX, X, grd);
    for (int c = 0; c < 3; ++c) {
      const float Ls = wt * X[c];
      gF0[c] += g[c] * Ls * beta[0];
      gb1 += g[c] * Ls * F0[c];
      gb2 += g[c] * Ls;
      gtl += (side ? 1.f : -1.f) * gLs[c] * X[c];
    }
  }
  for (int c = 0; c < 3; ++c) {
    g_metal += gF0[c] * (rho[c] - 0.04f);
    g_rho[c] += gF0[c] * metal;
  }
  float g_rc = 5.f * gtl;
  // BRDF table slopes
  float gnvc = 0.f;
  {
    const float* L = P.lut;
    for (int c = 0; c < 2; ++c) {
      const float t00 = L[(T.i0 * P.lut_nv + T.j0) * 2 + c];
      const float t01 = L[(T.i0 * P.lut_nv + T.j0 + 1) * 2 + c];
      const float t10 = L[((T.i0 + 1) * P.lut_nv + T.j0) * 2 + c];
      const float t11 = L[((T.i0 + 1) * P.lut_nv + T.j0 + 1) * 2 + c];
      const float dx = (1.f - T.fy) * (t01 - t00) + T.fy * (t11 - t10);
      const float dy = (1.f - T.fx) * (t10 - t00) + T.fx * (t11 - t01);
      const float gc = (c == 0) ? gb1 : gb2;
      gnvc += gc * dx * (float)(P.lut_nv - 1);
      g_rc += gc * dy * (float)(P.lut_r - 1);
    }
  }
  float gnv = (nv >= 0.f && nv <= 1.f) ? gnvc : 0.f;
  const float nhg = nh[0] * grd[0] + nh[1] * grd[1] + nh[2] * grd[2];
  gnv += 2.f * nhg;
  float gwo[3];
  for (int i = 0; i < 3; ++i) {
    g_nh[i] += 2.f * nv * grd[i] + gnv * wo[i];
    gwo[i] = -grd[i] + gnv * nh[i];
  }
  if (rough >= 0.f && rough <= 1.f) g_rough += g_rc;
  const float wg = wo[0] * gwo[0] + wo[1] * gwo[1] + wo[2] * gwo[2];
  for (int i = 0; i < 3; ++i) g_p[i] -= (gwo[i] - wo[i] * wg) / wl;
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
// rounded once.  The projected centre is stored relative to the integer corner
// of the pixel rectangle (a few pixels at most), so the pixel offset d that the
// raster forms is accurate to ~1e-7 px instead of the ~1e-4 px an FP32 centre
// near x = 1000 px would carry; thin (edge-on) ellipses amplify that error.
struct RasterGeoF {
  float x0r, y0r, Qxx, Qxy2, Qyy, a3, b3, nf;
};
__device__ inline void raster_geometry_f64(const float pf[3], const float nf_[3], const float tf[3],
                                           float su_, float sv_, const ViewDev& v, float sigma_,
                                           int il, int jl, RasterGeoF& out) {
  const double n0 = nf_[0], n1 = nf_[1], n2 = nf_[2];
  const double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  const double nh[3] = {n0 / nn, n1 / nn, n2 / nn};
  const double d = tf[0] * nh[0] + tf[1] * nh[1] + tf[2] * nh[2];
  double g[3] = {tf[0] - d * nh[0], tf[1] - d * nh[1], tf[2] - d * nh[2]};
  const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  const double uh[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
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
  const double z = cp[2], mx = cp[0] / z, my = cp[1] / z;
  const double fx = v.fx, fy = v.fy;
  const double x0 = fx * mx + (double)v.cx, y0 = fy * my + (double)v.cy;
  const double M11 = fx * (up[0] - mx * up[2]) / z, M12 = fx * (vp[0] - mx * vp[2]) / z;
  const double M21 = fy * (up[1] - my * up[2]) / z, M22 = fy * (vp[1] - my * vp[2]) / z;
  const double g1 = up[2] / z, g2 = vp[2] / z;
  const double dm = M11 * M22 - M12 * M21;
  const double detA = dm * dm;
  const double K11 = M11 * M11 + M12 * M12, K12 = M11 * M21 + M12 * M22, K22 = M21 * M21 + M22 * M22;
  const double detB = detA + sigma * (K11 + K22) + sigma * sigma;
  out.x0r = (float)(x0 - (double)il);
  out.y0r = (float)(y0 - (double)jl);
  out.Qxx = (float)((K22 + sigma) / detB);
  out.Qxy2 = (float)(-2.0 * K12 / detB);
  out.Qyy = (float)((K11 + sigma) / detB);
  out.nf = (float)sqrt(detA / detB);
  out.a3 = (float)((g2 * M21 - g1 * M22) / dm);
  out.b3 = (float)((M12 * g1 - M11 * g2) / dm);
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

struct PPtrs { const float* p[7]; };

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
//   the records of one scene.  The adjoint of the split-sum colour gives
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

__global__ void __launch_bounds__(kBackwardThreads, 1) shade_backward_kernel(
    PPtrs PP, long long N, const ViewDev* __restrict__ views, SceneViews sv, Params prm,
    const float* __restrict__ grad, float* __restrict__ sg, LocalMaps lm, float* __restrict__ partial) {
  extern __shared__ float sm[];
  for (int i = threadIdx.x; i < lm.total; i += blockDim.x) sm[i] = 0.f;
  __syncthreads();
  const long long n_rec = (long long)sv.n * sv.n_surf;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_rec;
       i += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(i / sv.n_surf);
    const long long local = i - (long long)k * sv.n_surf;
    const ViewDev& v = views[sv.idx[k]];
    const long long r = v.rec_off + local, s = sv.surf_off + local;
    float gr[12];
    if (!record_has_grad(grad, r, gr)) continue;
    // a record with a gradient was rasterised, hence kept by the cull; the
    // shading needs only the position and the unit normal
    const float p[3] = {PP.p[0][s], PP.p[0][N + s], PP.p[0][2 * N + s]};
    const float n[3] = {PP.p[1][s], PP.p[1][N + s], PP.p[1][2 * N + s]};
    const float nn = sqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const float nh[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
    const float rho[3] = {PP.p[4][s], PP.p[4][N + s], PP.p[4][2 * N + s]};
    float gp[3] = {0.f, 0.f, 0.f}, gnh[3] = {0.f, 0.f, 0.f}, grho[3] = {0.f, 0.f, 0.f};
    float grough = 0.f, gmetal = 0.f;
    const float gcol[3] = {gr[G_CR], gr[G_CG], gr[G_CB]};
    shade_backward(v, prm, p, nh, rho, PP.p[5][s], PP.p[6][s], gcol, sm, lm.off, gp, gnh, grho, grough,
                   gmetal);
    float4* out = reinterpret_cast<float4*>(sg + r * 12);
    out[0] = make_float4(gp[0], gp[1], gp[2], gnh[0]);
    out[1] = make_float4(gnh[1], gnh[2], grho[0], grho[1]);
    out[2] = make_float4(grho[2], grough, gmetal, 0.f);
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
    const float* __restrict__ recs, float* __restrict__ ss_out, int* __restrict__ vis_out) {
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
    if (!record_has_grad(grad, r, gr) && gtz == 0.f) continue;
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
    } else {
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
    float gdetB = -(gQxx * g.Qxx + gQxy * g.Qxy + gQyy * g.Qyy) / detB;
    float gdetA = 0.f;
    if (g.nf > 0.f) {
      gdetB += -gnf * g.nf / (2.f * detB);
      gdetA += gnf / (2.f * g.nf * detB);
    }
    float gK22 = gQxx / detB, gK12 = -gQxy / detB, gK11 = gQyy / detB;
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
    for (int j = 0; j < 3; ++j) gg[j] = (guh[j] - o.uh[j] * ug) / o.gn;
    // g = t - (t.n_hat) n_hat
    float ngg = o.nh[0] * gg[0] + o.nh[1] * gg[1] + o.nh[2] * gg[2];
    for (int j = 0; j < 3; ++j) {
      gt[j] += gg[j] - ngg * o.nh[j];
      gnh[j] += -o.d * gg[j] - ngg * t[j];
    }
    // n_hat = n / |n|
    float ng = o.nh[0] * gnh[0] + o.nh[1] * gnh[1] + o.nh[2] * gnh[2];
    for (int j = 0; j < 3; ++j) gn[j] += (gnh[j] - o.nh[j] * ng) / o.nn;
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
                                 float* sg, hipStream_t st) {
  if (n_surf <= 0 || n_scene_views <= 0) return hipSuccess;
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
  static bool lds_attr = false;  // allow the privatised levels beyond the default dynamic-LDS limit
  if (!lds_attr) {
    hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(&shade_backward_kernel),
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        kLocalMapFloats * (int)sizeof(float));
    if (ea != hipSuccess) return ea;
    lds_attr = true;
  }
  hipLaunchKernelGGL(shade_backward_kernel, dim3(nb), dim3(kBackwardThreads),
                     (size_t)local_total * sizeof(float), st, PP, N, views, sv, prm, grad, sg, lm,
                     partial);
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
                                    float* ss_out, int* vis_out, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  PPtrs PP;
  GPtrs GG;
  for (int k = 0; k < 7; ++k) { PP.p[k] = P[k]; GG.p[k] = G[k]; }
  hipLaunchKernelGGL(geometry_backward_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, PP, N,
                     views, n_views, prm, grad, sg, GG, recs, ss_out, vis_out);
  return hipGetLastError();
}

}  // namespace ss
